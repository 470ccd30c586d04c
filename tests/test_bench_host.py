"""Host-side arithmetic of bench.py (CPU): the multi-hit fit, the kernel-trace and counter
readers, the per-launch roofline, and the reduction of counter runs into the per-launch
summaries the bench line reads."""
from __future__ import annotations

import csv
import math

import pytest

import bench


def test_fit_multi_hit_recovers_the_law():
    N, t_inf, c, ms0 = 1 << 24, 0.8, 7.25, 0.17  # ps per hit, ps, ms per sweep at k = 0
    ms = {k: ms0 + (t_inf + c / k) * N * k * 1e-9 for k in (1, 4, 8)}
    r = bench.fit_multi_hit(ms, ms0, N)
    assert r["k"] == [1, 4, 8]
    assert math.isclose(r["t_inf_ps"], t_inf, rel_tol=1e-9)
    assert math.isclose(r["c_ps"], c, rel_tol=1e-9)
    assert r["max_rel_residual"] < 1e-9
    assert math.isclose(r["hits_per_ns_asymptotic"], 1e3 / t_inf, rel_tol=1e-9)


def _write_csv(path, rows, fields):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        w.writerows(rows)


def test_read_trace_csv_separates_isolated_dispatches(tmp_path):
    # queue 1: A at 0-10 us, B back to back at 10-20 us, A after a 5 us gap; queue 2: B alone
    rows = [
        {"Kernel_Name": "A", "Queue_Id": "1", "Start_Timestamp": 0, "End_Timestamp": 10000},
        {"Kernel_Name": "B", "Queue_Id": "1", "Start_Timestamp": 10000, "End_Timestamp": 20000},
        {"Kernel_Name": "A", "Queue_Id": "1", "Start_Timestamp": 25000, "End_Timestamp": 37000},
        {"Kernel_Name": "B", "Queue_Id": "2", "Start_Timestamp": 1000, "End_Timestamp": 4000},
    ]
    p = tmp_path / "kernel_trace.csv"
    _write_csv(p, rows, list(rows[0]))
    out, iso = bench.read_trace_csv(str(p))
    assert out == {"A": [10.0, 12.0], "B": [3.0, 10.0]}
    # the first dispatch of a queue has no predecessor; only A's second follows a gap
    assert iso == {"A": [12.0]}
    out, iso = bench.read_trace_csv(str(p), isolated_gap_us=0.0)
    assert iso == {"B": [10.0], "A": [12.0]}


def test_read_counter_csv_filters_by_counter(tmp_path):
    rows = [{"Kernel_Name": "K", "Counter_Name": "FETCH_SIZE", "Counter_Value": "10"},
            {"Kernel_Name": "K", "Counter_Name": "WRITE_SIZE", "Counter_Value": "4"},
            {"Kernel_Name": "K", "Counter_Name": "FETCH_SIZE", "Counter_Value": "12"}]
    p = tmp_path / "c.csv"
    _write_csv(p, rows, list(rows[0]))
    assert bench.read_counter_csv(str(p), "FETCH_SIZE") == {"K": [10.0, 12.0]}
    assert bench.read_counter_csv(str(p), "WRITE_SIZE") == {"K": [4.0]}


def test_kernel_roofline_counts_36_bytes_per_site_phase():
    N = 1 << 24
    r = bench.kernel_roofline(4, {"mean_ms": 0.25, "count": 3}, N, counted=False)
    nbytes = 1.5 * N * 36.0  # an over-relaxation phase and half a Metropolis phase
    assert r["bytes_per_launch"] == nbytes
    assert math.isclose(r["achieved"], nbytes / 0.25e-3 / 1e9)
    assert math.isclose(r["frac"], r["achieved"] / 8000.0)
    assert r["kernel"] == "phase_mc_kernel<float, MetropolisFull>"
    assert r["traffic"] is None
    p = bench.kernel_roofline(1, {"mean_ms": 0.1, "count": 1}, N, counted=False, brief=True)
    assert p["bytes_per_launch"] == 0.5 * N * 36.0 and "traffic" not in p


def test_reduce_counters_scales_by_the_copy(tmp_path, monkeypatch):
    """A 1 GiB copy that FETCH_SIZE reads as half its size sets the fetch scale to 2;
    the summary's bytes, issue rate and trace means follow, and the bench reads them back
    only while the sources hash to the stored value."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "source_hash", lambda name: "abc")
    name = "phase_mc"
    kname = "void hsg::phase_mc_kernel<float, (hsg::PassMode)3>(args)"
    copy = "__amd_rocclr_copyBuffer"
    f_rows = [{"Kernel_Name": copy, "Counter_Name": "FETCH_SIZE", "Counter_Value": 524288},
              {"Kernel_Name": kname, "Counter_Name": "FETCH_SIZE", "Counter_Value": 1000},
              {"Kernel_Name": kname, "Counter_Name": "FETCH_SIZE", "Counter_Value": 3000}]
    w_rows = [{"Kernel_Name": copy, "Counter_Name": "WRITE_SIZE", "Counter_Value": 1048576},
              {"Kernel_Name": kname, "Counter_Name": "WRITE_SIZE", "Counter_Value": 500}]
    i_rows = [{"Kernel_Name": kname, "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": 512000},
              {"Kernel_Name": kname, "Counter_Name": "GRBM_GUI_ACTIVE", "Counter_Value": 8000}]
    t_rows = [{"Kernel_Name": kname, "Queue_Id": "0", "Start_Timestamp": 0, "End_Timestamp": 200000},
              {"Kernel_Name": kname, "Queue_Id": "0", "Start_Timestamp": 300000,
               "End_Timestamp": 520000}]
    for fn, rows in (("f.csv", f_rows), ("w.csv", w_rows), ("i.csv", i_rows), ("t.csv", t_rows)):
        _write_csv(tmp_path / fn, rows, list(rows[0]))
    bench.reduce_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                          str(tmp_path / "i.csv"), str(tmp_path / "t.csv"))
    kv = bench.counter_summary(name)
    assert kv is not None
    assert float(kv["fetch_scale"]) == 2.0 and float(kv["write_scale"]) == 1.0
    assert float(kv["fetch_bytes_per_launch"]) == 2000 * 1024 * 2.0
    assert float(kv["write_bytes_per_launch"]) == 500 * 1024
    # 512000 wave-instructions over 256 CUs x 1000 cycles (8000 summed over 8 XCDs)
    assert float(kv["valu_insts_per_cu_cycle"]) == pytest.approx(2.0)
    assert float(kv["trace_mean_us"]) == pytest.approx(210.0)
    assert float(kv["trace_isolated_mean_us"]) == pytest.approx(220.0)
    assert float(kv["algorithmic_bytes_per_launch"]) == (1 << 24) * 1.5 * 36.0
    r = bench.kernel_roofline(4, {"mean_ms": 0.25, "count": 1}, 1 << 24, counted=True)
    assert r["traffic"] == 2000 * 1024 * 2.0 + 500 * 1024
    assert r["vector_issue"]["valu_wave_insts_per_launch"] == 512000
    assert r["kernel_ms_rocprofv3"] == pytest.approx(0.21)
    monkeypatch.setattr(bench, "source_hash", lambda name: "changed")
    assert bench.counter_summary(name) is None
