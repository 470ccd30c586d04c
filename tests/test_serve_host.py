"""Host logic of the served form (no GPU): the request stream, the arena allocator,
request validation and the latency statistics."""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import pytest

from paper_1006_2566_amd import serve as S


def test_poisson_trace_distributions():
    tr = S.poisson_trace(n=20000, rate=200.0, seed=3)
    arr = np.array([r.arrival for r in tr])
    gaps = np.diff(np.concatenate([[0.0], arr]))
    assert abs(gaps.mean() - 1 / 200) < 4 * (1 / 200) / math.sqrt(len(gaps))
    assert abs(np.std(gaps) / gaps.mean() - 1) < 0.05  # exponential: cv = 1
    Ls = np.array([r.L for r in tr])
    assert set(np.unique(Ls)) == {8, 16, 32, 64, 96}
    for L in (8, 16, 32, 64, 96):
        assert abs((Ls == L).mean() - 0.2) < 0.02
    sw = np.array([r.sweeps for r in tr])
    assert sw.min() >= 100 and sw.max() <= 10000
    # log-uniform: log(sweeps) uniform on [log 100, log 10000]
    u = (np.log(sw) - math.log(100)) / (math.log(10000) - math.log(100))
    assert abs(u.mean() - 0.5) < 0.01 and abs(u.var() - 1 / 12) < 0.005
    T = np.array([r.T for r in tr])
    assert 0.1 <= T.min() and T.max() <= 1.0
    assert set(np.unique([r.k for r in tr])) == {1, 4}
    assert [r.seed for r in tr[:3]] == [1000, 1001, 1002]


def test_arena_first_fit_and_coalescing():
    a = S.Arena(1000, align=10)
    x = a.alloc(95)    # rounded to 100
    y = a.alloc(300)
    z = a.alloc(200)
    assert (x, y, z) == (0, 100, 400)
    assert a.alloc(500) is None and a.used == 600
    a.release(y, 300)
    assert a.alloc(250) == 100     # first fit reuses the hole
    a.release(100, 250)
    a.release(x, 95)
    a.release(z, 200)
    assert a.free == [(0, 1000)] and a.used == 0


def test_latency_stats():
    res = [S.Result(i, 0.0, np.zeros(3), arrival=0.0, admitted=0.0, finished=float(i))
           for i in range(1, 101)]
    st = S.latency_stats(res)
    assert st["n"] == 100 and st["p50_s"] == pytest.approx(50.5) and st["max_s"] == 100
    assert st["p99_s"] == pytest.approx(99.01)


def test_latency_stats_count_completed_requests_only():
    res = [S.Result(i, 0.0, np.zeros(3), arrival=0.0, admitted=0.0, finished=float(i))
           for i in range(1, 11)]
    res.append(S.Result(99, float("nan"), np.full(3, np.nan), 5.0, 0.0, 0.0, status="cancelled"))
    res.append(S.Result(98, float("nan"), np.full(3, np.nan), 5.0, 0.0, 0.0,
                        status="rejected: L=3 must be even"))
    st = S.latency_stats(res)
    assert st["n"] == 10 and st["cancelled"] == 1 and st["rejected"] == 1
    assert st["max_s"] == 10


def test_request_problem():
    ok = S.Request(rid=0, seed=1, L=16, T=0.5, sweeps=10, k=4)
    cap = 3 * 16 ** 3
    assert S.request_problem(ok, cap) is None
    assert S.request_problem(dataclasses.replace(ok, T=float("inf")), cap) is None  # beta = 0
    assert S.request_problem(dataclasses.replace(ok, sweeps=0), cap) is None
    bad = {"L": [3, 0, S.BATCH_L_MAX + 2], "k": [0, 70000], "T": [0.0, -1.0, float("nan")],
           "sweeps": [-1], "seed": [-1, 2 ** 64]}
    for field, values in bad.items():
        for v in values:
            assert S.request_problem(dataclasses.replace(ok, **{field: v}), 10 ** 9), (field, v)
    # the footprint against the arena, in its 64-element blocks
    assert S.request_problem(ok, cap - 1) is not None
    small = dataclasses.replace(ok, L=2)  # 24 elements take one block of 64
    assert S.request_problem(small, 64) is None and S.request_problem(small, 63) is not None


def test_autotune_pick_caches_the_fastest(tmp_path):
    from paper_1006_2566_amd import autotune as A
    path = str(tmp_path / "tune.json")
    calls = []

    def measure(c):
        calls.append(c)
        return {64: 3.0, 128: 1.0, 256: 2.0}[c]
    assert A.pick("k1", [64, 128, 256], measure, path=path, dev="gfxTEST") == 128
    assert calls == [64, 128, 256]
    # cached: no new measurements, even with another candidate order
    assert A.pick("k1", [256, 128, 64], measure, path=path, dev="gfxTEST") == 128
    assert len(calls) == 3
    # a cached choice that is no longer a candidate is re-measured
    assert A.pick("k1", [64, 256], measure, path=path, dev="gfxTEST") == 256
    # retune forces new measurements; other devices keep their own entries
    A.pick("k1", [64, 128], measure, path=path, dev="gfxTEST", retune=True)
    A.pick("k1", [64, 256], measure, path=path, dev="gfxOTHER")
    data = A.load_cache(path)
    assert data["gfxTEST"]["k1"]["choice"] == 128 and data["gfxOTHER"]["k1"]["choice"] == 256
    assert set(data["gfxTEST"]["k1"]["ms"]) == {"64", "128"}


def test_autotune_cache_tolerates_garbage(tmp_path):
    from paper_1006_2566_amd import autotune as A
    path = tmp_path / "tune.json"
    path.write_text("{not json")
    assert A.load_cache(str(path)) == {}
    assert A.pick("k", [1, 2], lambda c: float(c), path=str(path), dev="x") == 1
