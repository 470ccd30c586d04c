"""Benchmark: checkerboard Monte Carlo sweeps of the 3D Heisenberg spin glass on one
MI355X, L = 256 (16.8M spins), binary32 spins and couplings, Gaussian couplings.

One step = one full sweep of the lattice: the Metropolis phase with k hits per
site (colour-0 pass, colour-1 pass), one over-relaxation phase (two passes),
renormalisation every 10 sweeps, and the tracked binary64 energy folded once per
call.  The headline is k = 4; the same line also reports k = 1 and k = 8.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Prints ONE JSON line.  value = spin updates per ns, counting each Metropolis hit
and each over-relaxation step at a site as one update: N * (k + n_or) per sweep.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spin updates/ns at L=256 FP32 (k=1,4,8) + %HBM roofline; batched p50/p99 latency"
HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
BYTES_PER_SITE_PHASE = 36.0  # binary32: read spin (12) + 3 bonds (12), write spin (12)
# the other byte models per site-phase: a phase as two colour passes, each reading all six
# coupling planes, its own spins and the other colour's (60 B); every neighbour and bond
# read from memory at every site (120 B)
BYTE_MODELS = {"algorithmic_36B": 36.0, "two_pass_60B": 60.0, "naive_120B": 120.0}
_COMMON_SOURCES = ("paper_1006_2566_amd/csrc/hsg_site.h", "paper_1006_2566_amd/csrc/hsg_device.h",
                   "paper_1006_2566_amd/csrc/hsg_internal.h")
# The kernels that can dominate the headline sweep: the binary32 Metropolis colour pass,
# and the launch of the over-relaxation phase with the next sweep's colour-0 Metropolis
# pass (HSG_PHASE_MC).  Each has its counter summary, valid while its sources are those
# the counters were taken from.
DOMINANT = {
    "metropolis_pass": {
        # k a multiple of four: the instantiation whose hit groups are all complete
        "kernel": "colour_pass_kernel<float, MetropolisFull>",
        "trace_name": "colour_pass_kernel<float, (hsg::PassMode)3, false>",
        "sources": _COMMON_SOURCES + ("paper_1006_2566_amd/csrc/kernels_sweep.hip",),
        "traffic_file": "profiles/traffic_metropolis_pass_L256_f32.txt",
        "title": "one Metropolis colour pass",
        "sites": 0.5,  # updated sites per launch, in units of N
    },
    "phase_mc": {
        "kernel": "phase_mc_kernel<float, MetropolisFull>",
        "trace_name": "phase_mc_kernel<float, (hsg::PassMode)3>",
        "sources": _COMMON_SOURCES + ("paper_1006_2566_amd/csrc/kernels_phase.hip",),
        "traffic_file": "profiles/traffic_phase_mc_L256_f32.txt",
        "title": "one over-relaxation phase with the next colour-0 Metropolis pass",
        # an over-relaxation phase (every site once) and half a Metropolis phase (the
        # colour-0 sites): 1.5 site-phases per site
        "sites": 1.5,
    },
    "phase": {
        "kernel": "phase_kernel<float>",
        "trace_name": "phase_kernel<float>(",
        "sources": _COMMON_SOURCES + ("paper_1006_2566_amd/csrc/kernels_phase.hip",),
        "traffic_file": "profiles/traffic_phase_L256_f32.txt",
        "title": "one over-relaxation phase",
        "sites": 1.0,
    },
}
# launch kinds of hsg_sweep_timed -> (dominant-kernel entry, site-phases per launch in
# units of N): a colour pass updates half the sites (half a phase)
LAUNCH_ROOFLINE = {1: ("metropolis_pass", 0.5), 2: (None, 0.5), 3: ("phase", 1.0),
                   4: ("phase_mc", 1.5)}
CLOCK_GHZ = 2.4  # MI355X peak engine clock
N_CU = 256


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--L", type=int, default=256)
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--also-k", default="1,8")
    ap.add_argument("--n-or", type=int, default=1)
    ap.add_argument("--T", type=float, default=0.3)
    ap.add_argument("--renorm-every", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--flags", type=int, default=None,
                    help="hsg_sweep flags for the timed sweeps (default: the library's choice)")
    ap.add_argument("--batch-cycles", type=int, default=2,
                    help="timed cycles (100 sweeps each) of the batched tempering workload; "
                         "0 skips that leg")
    ap.add_argument("--batch-threads", type=int, default=0,
                    help="workgroup size of the batched sweep (0 = autotuned)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="requests of the served stream (0 skips that leg)")
    ap.add_argument("--no-serve-load-sweep", dest="serve_load_sweep", action="store_false",
                    help="skip the served streams at 100 and 50 requests per second")
    ap.add_argument("--serve-budget-mb", type=int, default=8192,
                    help="device memory for resident lattices of the served stream")
    ap.add_argument("--serve-step", type=int, default=16, help="sweeps per scheduling step")
    ap.add_argument("--serve-tile", type=int, default=0,
                    help="sites per tile of the served passes (0 = autotuned)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library defaults instead of timing candidate launch shapes")
    ap.add_argument("--no-binary64", action="store_true",
                    help="skip timing the headline sweep with binary64 spins")
    ap.add_argument("--no-heat-bath", action="store_true",
                    help="skip timing the headline sweep with heat-bath draws")
    ap.add_argument("--no-large-L", dest="large_L", action="store_false",
                    help="skip the L = 512 row")
    ap.add_argument("--no-observables", action="store_true",
                    help="skip timing the Fourier-overlap records (chi_SG, xi inputs)")
    ap.add_argument("--counters", action="store_true",
                    help="short run for hardware-counter collection: one 1 GiB device copy "
                         "(calibrates FETCH_SIZE / WRITE_SIZE), then 4 sweeps of the headline "
                         "configuration; prints no JSON")
    ap.add_argument("--reduce-counters", nargs="+", metavar="CSV",
                    help="FETCH_CSV WRITE_CSV [ISSUE_CSV[,ISSUE_CSV...] [TRACE_CSV]]: turn the "
                         "counter_collection.csv files of a FETCH_SIZE and a WRITE_SIZE run of "
                         "--counters (and optionally of an SQ_INSTS_VALU + GRBM_GUI_ACTIVE run "
                         "and the kernel_trace.csv of a --kernel-trace run of the same command) "
                         "into the per-launch summaries of the kernels the run dispatched ("
                         + ", ".join(d["traffic_file"] for d in DOMINANT.values()) + "), then exit")
    return ap.parse_args()


def source_hash(name: str) -> str:
    """sha256 over the sources a dominant-kernel candidate is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for rel in DOMINANT[name]["sources"]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_counter_csv(path, counter=None):
    """{kernel name: [value per dispatch]} of one counter from rocprofv3's CSV (the only
    counter of the file, or the one named)."""
    import csv
    out = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if counter is not None and row.get("Counter_Name") != counter:
                continue
            out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def read_trace_csv(path, isolated_gap_us=2.0):
    """{kernel name: [duration in us per dispatch]} from rocprofv3's kernel_trace.csv, and
    the same for the dispatches that start at least isolated_gap_us after the previous
    dispatch of the queue ended.  The latter are the launches hsg_sweep_timed brackets
    with events (their markers leave such a gap); under the profiler, launches that follow
    each other with no gap run longer than the same launches without it, which is not so
    without the profiler (the plain sweep time equals the sum of the event-timed launches
    there)."""
    import csv
    out, isolated = {}, {}
    with open(path, newline="") as f:
        rows = sorted(csv.DictReader(f), key=lambda r: int(r["Start_Timestamp"]))
    prev_end = {}
    for row in rows:
        q = row.get("Queue_Id", "")
        start, end = int(row["Start_Timestamp"]), int(row["End_Timestamp"])
        d = (end - start) * 1e-3
        out.setdefault(row["Kernel_Name"], []).append(d)
        if q in prev_end and (start - prev_end[q]) * 1e-3 >= isolated_gap_us:
            isolated.setdefault(row["Kernel_Name"], []).append(d)
        prev_end[q] = end
    return out, isolated


# vector instruction classes counted beside SQ_INSTS_VALU for the issue mix
VALU_MIX = ("SQ_INSTS_VALU_INT32", "SQ_INSTS_VALU_INT64", "SQ_INSTS_VALU_FMA_F32",
            "SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_TRANS_F32")


def reduce_counters(fetch_csv, write_csv, issue_csv=None, trace_csv=None):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of each dominant-kernel candidate the
    run dispatched, each scaled by what the same counter reads for the 1 GiB device copy
    of the --counters run; with issue_csv, its vector wave-instructions per launch and per
    compute unit and cycle (SQ_INSTS_VALU / (256 x GRBM_GUI_ACTIVE / 8 XCDs)); with
    trace_csv, its mean kernel-trace duration."""
    fetch, write = read_counter_csv(fetch_csv), read_counter_csv(write_csv)
    issue = {}
    for path in (issue_csv.split(",") if issue_csv else []):  # one or more counter runs
        for c in ("SQ_INSTS_VALU", "GRBM_GUI_ACTIVE") + VALU_MIX:
            got = read_counter_csv(path, c)
            if got:
                issue[c] = got
    trace, trace_iso = read_trace_csv(trace_csv) if trace_csv else ({}, {})

    def pick(d, key):
        names = [n for n in d if key(n)]
        if len(names) > 1:
            raise SystemExit(f"expected one kernel, found {names}")
        return d[names[0]] if names else None

    def mean(v):
        return sum(v) / len(v)

    copy_f = pick(fetch, lambda n: "copy" in n.lower())
    copy_w = pick(write, lambda n: "copy" in n.lower())
    if copy_f is None or copy_w is None:
        raise SystemExit("no device copy in the counter runs")
    gib_kib = float(1 << 20)
    f_scale = gib_kib / max(copy_f)
    w_scale = gib_kib / max(copy_w)
    written = 0
    for name, d in DOMINANT.items():
        match = lambda n, d=d: d["trace_name"] in n  # noqa: E731
        k_f = pick(fetch, match)
        k_w = pick(write, match)
        if k_f is None or k_w is None:
            continue
        f_b = mean(k_f) * 1024 * f_scale
        w_b = mean(k_w) * 1024 * w_scale
        lines = [
            f"# HBM traffic of {d['title']} ({d['kernel']}), L=256 binary32, k=4",
            "# commands: rocprofv3 --pmc FETCH_SIZE -d <dir> -o run --output-format csv -- "
            "python bench.py --counters   (then the same with WRITE_SIZE, and with "
            "SQ_INSTS_VALU GRBM_GUI_ACTIVE + the SQ_INSTS_VALU_* classes; and "
            "rocprofv3 --kernel-trace --output-format csv)",
            "#           python bench.py --reduce-counters <fetch csv> <write csv> [<issue csv> "
            "[<kernel_trace csv>]]",
            f"copy_fetch_kib={max(copy_f):.0f} fetch_scale={f_scale:.4f}",
            f"copy_write_kib={max(copy_w):.0f} write_scale={w_scale:.4f}",
            f"dispatches={len(k_f)}",
            f"fetch_bytes_per_launch={f_b:.0f}",
            f"write_bytes_per_launch={w_b:.0f}",
            f"algorithmic_bytes_per_launch={(1 << 24) * d['sites'] * BYTES_PER_SITE_PHASE:.0f}",
        ]
        v = pick(issue.get("SQ_INSTS_VALU", {}), match)
        g = pick(issue.get("GRBM_GUI_ACTIVE", {}), match)
        if v:
            lines.append(f"valu_insts_per_launch={mean(v):.0f}")
            if g:
                lines.append(f"valu_insts_per_cu_cycle={mean(v) / (N_CU * mean(g) / 8):.3f}")
            mix = []
            for c in VALU_MIX:
                x = pick(issue.get(c, {}), match)
                if x:
                    mix.append(f"{c[len('SQ_INSTS_VALU_'):].lower()}:{mean(x) / mean(v):.3f}")
            if mix:
                lines.append("valu_mix=" + ",".join(mix))
        t = pick(trace, match)
        if t:
            lines.append(f"trace_dispatches={len(t)} trace_mean_us={mean(t):.2f}")
            ti = pick(trace_iso, match)
            if ti:
                lines.append(f"trace_isolated_dispatches={len(ti)} "
                             f"trace_isolated_mean_us={mean(ti):.2f}")
        lines.append(f"source_hash={source_hash(name)}")
        with open(os.path.join(ROOT, d["traffic_file"]), "w") as f:
            f.write("\n".join(lines) + "\n")
        print("\n".join(lines))
        written += 1
    if not written:
        raise SystemExit("none of the dominant-kernel candidates was dispatched")


def counter_summary(name: str) -> dict | None:
    """key=value pairs of a dominant-kernel candidate's committed counter summary, or None
    when it is missing or its sources changed since the counters were taken."""
    path = os.path.join(ROOT, DOMINANT[name]["traffic_file"])
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                for item in line.split():
                    k, _, v = item.partition("=")
                    kv[k] = v
    return kv if kv.get("source_hash") == source_hash(name) else None


def note(msg: str) -> None:
    """A progress line on stderr (the JSON result is the last line on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_sweeps(lat, torch, *, T, k, n_or, R, steps, warmup, flags=0):
    """Average ms per sweep over `steps` sweeps, HIP events on the launch stream."""
    lat.sweep(T=T, k=k, n_or=n_or, renorm_every=R, n_sweeps=warmup, flags=flags)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    lat.sweep(T=T, k=k, n_or=n_or, renorm_every=R, n_sweeps=steps, flags=flags)
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / steps


def binary64_leg(hsg, args, torch, flags):
    """The headline sweep with binary64 spins and couplings (the large-lattice
    configuration compares binary32 with binary64): same L, k, n_or and T, with the
    library's traversal for binary64."""
    L = args.L
    lat = hsg.Lattice(L, torch.float64, seed=1)
    steps = max(5, args.steps // 5)
    ms = time_sweeps(lat, torch, T=args.T, k=args.k, n_or=args.n_or, R=args.renorm_every,
                     steps=steps, warmup=2, flags=flags)
    del lat
    torch.cuda.empty_cache()
    return {"dtype": "f64", "steps": steps, "ms_per_step": ms, "flags": flags,
            "spin_updates_per_ns": L ** 3 * (args.k + args.n_or) / (ms * 1e6)}


# The paper's Table 2 (over-relaxation only, L = 128, binary32, 100 iterations): its GPU
# figures, ns per spin update, with the GPUs of its hardware table (context, other hardware)
PAPER_TABLE2_NS = {"GTX 480, TEXT (its best)": 0.63, "GTX 480, GM": 0.66,
                   "GTX 480, SM4P": 0.86, "Tesla C1060, TEXT": 1.8, "Tesla C1060, GM": 1.9}


def paper_workload_leg(hsg, torch):
    """The paper's benchmark workload on this GPU: over-relaxation sweeps only (both
    colours, no renormalisation) of an L = 128 binary32 lattice with Gaussian couplings,
    100 iterations after 5 warm-up ones, the library's default traversal for that L."""
    L, n = 128, 100
    lat = hsg.Lattice(L, torch.float32, seed=1)
    flags = hsg.default_flags(L, torch.float32)
    ms = time_sweeps(lat, torch, T=1.0, k=0, n_or=1, R=0, steps=n, warmup=5, flags=flags)
    ns_per_update = ms * 1e6 / L ** 3
    del lat
    return {"workload": "over-relaxation only, L=128, binary32, 100 iterations (the paper's "
                        "Table 2 benchmark)", "flags": flags, "ms_per_sweep": ms,
            "ns_per_update": ns_per_update, "updates_per_ns": 1.0 / ns_per_update,
            "paper_ns_per_update": PAPER_TABLE2_NS,
            "note": "the paper's figures are other hardware: context, not the target"}


def heat_bath_leg(hsg, lat, torch, args, flags):
    """The headline sweep with a heat-bath draw in place of the Metropolis hits (same
    traversal).  A heat-bath draw does not depend on the spin it replaces, so a site
    takes one draw per Monte Carlo phase (k draws would leave the last): one update per
    site and phase.  The heat-bath colour pass is timed from the launches of the sweep
    (hsg_sweep_timed)."""
    N = lat.L ** 3
    steps = max(10, args.steps // 2)
    f = flags | hsg.HSG_HEAT_BATH
    ms = time_sweeps(lat, torch, T=args.T, k=1, n_or=args.n_or, R=args.renorm_every,
                     steps=steps, warmup=2, flags=f)
    launches = traced_launches(hsg, lat, T=args.T, k=1, n_or=args.n_or, R=args.renorm_every,
                               n=steps, flags=f)
    out = {"draws_per_site_phase": 1, "steps": steps, "ms_per_step": ms, "flags": f,
           "spin_updates_per_ns": N * (1 + args.n_or) / (ms * 1e6),
           "launches": {hsg.LAUNCH_NAMES[kd]: v for kd, v in launches.items()}}
    if hsg.LAUNCH_MC_PASS in launches:
        ms_pass = launches[hsg.LAUNCH_MC_PASS]["mean_ms"]
        out["pass"] = {"kernel": "colour_pass_kernel<float, HeatBath>", "kernel_ms": ms_pass,
                       "draws_per_ns": N / 2 / (ms_pass * 1e6)}
    return out


def observables_leg(hsg, lat, torch, steps):
    """The spin-glass observables of a replica pair at the headline size: the
    Fourier-overlap record (hsg_overlap_fourier), HBM-bound -- both replicas' spins are
    read once, 2 x 3 x 4 bytes per site; the rest is 63 binary64 sums per site."""
    L = lat.L
    other = hsg.Lattice(L, torch.float32, seed=2)
    out = torch.empty(hsg.FOURIER_VALUES, dtype=torch.float64, device="cuda")
    for _ in range(3):
        lat.overlap_fourier(other, out=out)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(steps):
        lat.overlap_fourier(other, out=out)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    nbytes = 2 * 3 * 4 * L ** 3
    gbs = nbytes / (ms * 1e-3) / 1e9
    rec = out.cpu().tolist()
    return {"entry": "hsg_overlap_fourier", "L": L, "dtype": "f32",
            "kernels": "fourier_partials_kernel<float> + fourier_finish_kernel",
            "us_per_call": ms * 1e3, "bound": "hbm", "bytes_per_call": nbytes,
            "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS,
            "N_q2_0": rec[63] * L ** 3, "N_q2_kmin": rec[64] * L ** 3}


def batched_leg(args, torch):
    """Parallel-tempering workload: 256 disorder samples, L uniform in {16,24,32,48},
    2 replicas x 24 geometric temperatures in [0.12, 0.5], binary32, Metropolis k=4,
    an exchange round every 10 sweeps and the binary64 overlap of the two replicas in
    every slot every 100 sweeps, all in one captured graph per 100 sweeps.  Compared
    with the same kind of lattices advanced by plain per-lattice hsg_sweep calls."""
    import numpy as np

    import paper_1006_2566_amd as hsg
    from paper_1006_2566_amd import batch as B

    specs, ladders, betas, pairs = B.pt_workload()
    b = B.Batch(specs, threads=args.batch_threads or 256)
    if not args.batch_threads and not args.no_autotune:
        from paper_1006_2566_amd import autotune
        autotune.batch_threads(b)
    pt = B.Tempering(b, ladders, betas, seed=1)
    runner = B.PTRunner(b, pt, pairs, sweeps_per_exchange=10, exchanges_per_measure=10)
    runner.run_cycle()  # eager first cycle, then the graph is captured
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(args.batch_cycles):
        runner.run_cycle()
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    sites = float(sum(sp.L ** 3 for sp in specs))
    sweeps = args.batch_cycles * runner.sweeps_per_cycle
    upd = sites * 4 * sweeps / (ms * 1e6)
    # the same lattices through plain per-lattice launches: one sample of each L,
    # all 48 chains, 2 sweeps each, one lattice at a time, no graph
    Ls = sorted({sp.L for sp in specs})
    lats = []
    for L in Ls:
        for c in range(48):
            lats.append(hsg.Lattice(L, torch.float32, seed=7 + 131 * c + L))
    for lat in lats:
        lat.sweep(T=0.3, k=4, n_sweeps=1)
    torch.cuda.synchronize()
    t0.record(stream)
    for lat in lats:
        lat.sweep(T=0.3, k=4, n_sweeps=2)
    t1.record(stream)
    torch.cuda.synchronize()
    ms_plain = t0.elapsed_time(t1)
    upd_plain = sum(l.N for l in lats) * 4 * 2 / (ms_plain * 1e6)
    acc = pt.accepted.sum().item() / max(1, int(pt.round.item())) / pt.n_ladders
    # each chain's tracked energy (binary64 sums of its binary32 energy changes) against a
    # binary64 recomputation of its final binary32 state, after the timed cycles
    E_tr = b.energies().double().cpu().numpy()
    E_re = b.energies(recompute=True).double().cpu().numpy()
    rel = np.abs(E_tr - E_re) / np.maximum(np.abs(E_re), 1e-300)
    return {"workload": "256 samples x 2 replicas x 24 temperatures (12288 chains, "
                        f"{sites:.3g} spins), L in {{16,24,32,48}}, binary32, k=4, exchange "
                        "every 10 sweeps, overlap every 100, one graph per 100 sweeps",
            "sweeps": sweeps, "ms": ms, "ms_per_sweep": ms / sweeps,
            "spin_updates_per_ns": upd,
            "plain_per_lattice_updates_per_ns": upd_plain,
            "speedup_vs_plain": upd / upd_plain,
            "exchange_acceptance_per_pair_round": acc,
            "energy_tracked_vs_binary64_recompute": {
                "chains": int(rel.size), "max_rel": float(rel.max()),
                "median_rel": float(np.median(rel))},
            "threads": b.threads}


def served_leg(args, torch):
    """Request stream: Poisson arrivals at 200 per second, L uniform in
    {8,16,32,64,96}, T uniform in [0.1,1], sweeps log-uniform in [100,10000], k in
    {1,4}, binary32, admitted by device-memory footprint, lattices resident between
    steps, continuous batching; latency = completion - arrival (wall clock).  The same
    kind of stream at 100 and 50 requests per second measures latency below saturation
    (offered load / delivered capacity = rho).  Baseline: the same requests one after
    another through plain per-lattice calls (initial state, sweeps with hsg_sweep,
    energy read back) -- every 10th request of the 200/s trace, a systematic sample of
    the whole trace."""
    import paper_1006_2566_amd as hsg
    from paper_1006_2566_amd import serve as S

    trace = S.poisson_trace(n=args.serve_requests, rate=200.0, seed=1)
    tile = args.serve_tile or 256
    if not args.serve_tile and not args.no_autotune:
        from paper_1006_2566_amd import autotune
        tile = autotune.serve_shape(trace[:64])["tile_sites"]

    def serve(tr):
        srv = S.Server(hbm_budget=args.serve_budget_mb << 20, n_slots=2048,
                       step_sweeps=args.serve_step, tile_sites=tile)
        srv.run([S.Request(rid=-1, seed=1, L=8, T=1.0, sweeps=2, k=1)], realtime=False)
        t0 = time.perf_counter()
        res = srv.run(tr, realtime=True)
        wall = time.perf_counter() - t0
        work = float(sum(r.L ** 3 * r.sweeps * r.k for r in tr))
        st = S.latency_stats(res)
        serve.results = res
        return {"requests": len(tr), "rate_per_s": len(tr) / tr[-1].arrival,
                "p50_latency_s": st["p50_s"], "p99_latency_s": st["p99_s"],
                "mean_latency_s": st["mean_s"], "wall_s": wall,
                "spin_updates_per_ns": work / (wall * 1e9),
                "offered_updates_per_ns": work / tr[-1].arrival / 1e9,
                "scheduler": {k: (round(v, 3) if isinstance(v, float) else v)
                              for k, v in srv.stats.items()}}

    main = serve(trace)
    served_E = {r.rid: r.E for r in serve.results}
    capacity = main["spin_updates_per_ns"]
    main["rho"] = main["offered_updates_per_ns"] / capacity
    sweep = {}
    if args.serve_load_sweep:
        for rate, n in ((100.0, max(50, args.serve_requests // 2)),
                        (50.0, max(25, args.serve_requests // 4))):
            r = serve(S.poisson_trace(n=n, rate=rate, seed=2))
            r["rho"] = r["offered_updates_per_ns"] / capacity
            sweep[f"{int(rate)}_per_s"] = {k: v for k, v in r.items() if k != "scheduler"}
            note(f"served at {rate:.0f}/s: p50 {r['p50_latency_s']:.3f} s, "
                 f"p99 {r['p99_latency_s']:.3f} s, rho {r['rho']:.2f}")
    sample = trace[::10]
    torch.cuda.synchronize()
    elapsed = 0.0
    err_re, err_served = [], []
    for r in sample:
        t1 = time.perf_counter()
        lat = hsg.Lattice(r.L, torch.float32, seed=r.seed)
        lat.sweep(T=r.T, k=r.k, n_or=0, n_sweeps=r.sweeps)
        E_tr = lat.energy().item()
        elapsed += time.perf_counter() - t1
        # not timed: the result's energy against a binary64 recomputation of the final
        # binary32 state, and the served run's result against this one
        E_re = lat.energy(recompute=True).item()
        err_re.append(abs(E_tr - E_re) / max(abs(E_re), 1e-300))
        err_served.append(abs(served_E[r.rid] - E_tr) / max(abs(E_re), 1e-300))
        del lat
    plain = sum(r.L ** 3 * r.sweeps * r.k for r in sample) / (elapsed * 1e9)
    return {"workload": f"{len(trace)} requests, Poisson 200/s, L in {{8,16,32,64,96}}, "
                        "T in [0.1,1], sweeps log-uniform [100,1e4], k in {1,4}, binary32",
            **{k: v for k, v in main.items() if k != "scheduler"},
            "plain_per_lattice_updates_per_ns": plain,
            "plain_sample": f"every 10th request of the trace ({len(sample)} requests)",
            "energy_error": {
                "results": len(sample),
                "tracked_vs_binary64_recompute_max_rel": max(err_re),
                "tracked_vs_binary64_recompute_median_rel": sorted(err_re)[len(err_re) // 2],
                "served_vs_alone_max_rel": max(err_served)},
            "speedup_vs_plain": capacity / plain, "budget_mb": args.serve_budget_mb,
            "step_sweeps": args.serve_step, "tile_sites": tile,
            "load_sweep": sweep, "scheduler": main["scheduler"]}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(args):
    """The CPU oracle, unchanged, on the host cores: the same L, k, n_or and T, as many
    whole sweeps as fit in about args.cpu_seconds (at least one) with every OpenMP
    thread, then one sweep on a single thread; and the paper's own workload (§4,
    Table 2: over-relaxation only, L = 128, binary32, 100 sweeps) on all threads and,
    for 10 sweeps, on one."""
    import numpy as np

    import oracle as O

    L = args.L
    threads = O.threads()
    spins, J = O.init(L, 1, np.float32)
    E = O.energy(L, spins, J)

    def run(n_max, seconds, sweep0=0, **kw):
        nonlocal E
        n, t0 = 0, time.perf_counter()
        while n < n_max:
            E = O.sweep(L, 1, spins, J, n_sweeps=1, sweep0=sweep0 + n, E=E, **kw)["E"]
            n += 1
            if time.perf_counter() - t0 >= seconds:
                break
        return n, time.perf_counter() - t0

    kw = dict(T=args.T, k=args.k, n_or=args.n_or, renorm_every=args.renorm_every)
    n, dt = run(1 << 30, args.cpu_seconds, **kw)
    per = L ** 3 * (args.k + args.n_or)
    O.set_threads(1)
    try:
        n1, dt1 = run(1, 0.0, sweep0=n, **kw)
        s128, J128 = O.init(128, 1, np.float32)
        t0 = time.perf_counter()
        O.sweep(128, 1, s128, J128, T=1.0, k=0, n_or=1, n_sweeps=10)
        or1 = 128 ** 3 * 10 / ((time.perf_counter() - t0) * 1e9)
    finally:
        O.set_threads(threads)
    t0 = time.perf_counter()
    O.sweep(128, 1, s128, J128, T=1.0, k=0, n_or=1, n_sweeps=100)
    orN = 128 ** 3 * 100 / ((time.perf_counter() - t0) * 1e9)
    return {"value": per * n / (dt * 1e9), "unit": "spin updates/ns", "cores": threads,
            "kind": "oracle",
            "sample": f"L={L} binary32, {n} sweep(s) of k={args.k} Metropolis + {args.n_or} "
                      f"over-relaxation, T={args.T}, {dt:.1f} s wall on {threads} OpenMP "
                      f"threads",
            "cpu_model": cpu_model(), "logical_cpus": os.cpu_count(),
            "single_thread": {"value": per * n1 / (dt1 * 1e9), "unit": "spin updates/ns",
                              "sample": f"{n1} sweep, {dt1:.1f} s"},
            "paper_workload": {
                "workload": "over-relaxation only, L=128, binary32 (the paper's Table 2 "
                            "benchmark)",
                "all_threads": {"updates_per_ns": orN, "ns_per_update": 1.0 / orN,
                                "threads": threads, "sweeps": 100},
                "single_thread": {"updates_per_ns": or1, "ns_per_update": 1.0 / or1,
                                  "sweeps": 10},
                "paper_i7_ns_per_update": {"1_thread_sse": 13.5, "8_threads_sse": 5.0}}}


def traced_launches(hsg, lat, *, T, k, n_or, R, n, flags) -> dict:
    """{launch kind: count, mean and total ms} over n sweeps through hsg_sweep_timed."""
    lat.sweep(T=T, k=k, n_or=n_or, renorm_every=R, n_sweeps=2, flags=flags)
    rec = lat.sweep_timed(T=T, k=k, n_or=n_or, renorm_every=R, n_sweeps=n, flags=flags,
                          capacity=16 * n + 16)
    out = {}
    for kd, ms in rec:
        d = out.setdefault(kd, {"count": 0, "total_ms": 0.0})
        d["count"] += 1
        d["total_ms"] += ms
    for d in out.values():
        d["mean_ms"] = d["total_ms"] / d["count"]
    return out


def kernel_roofline(kind: int, stats: dict, N: int, counted: bool, brief: bool = False) -> dict:
    """HBM roofline of one kind of launch: algorithmic bytes per launch (36 B per site-phase
    x the site-phases one launch performs) over its event-timed mean duration."""
    name, site_phases = LAUNCH_ROOFLINE[kind]
    nbytes = site_phases * N * BYTES_PER_SITE_PHASE
    ms = stats["mean_ms"]
    gbs = nbytes / (ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": gbs / HBM_PEAK_GBS, "kernel_ms": ms, "bytes_per_launch": nbytes,
           "site_phases_per_launch": site_phases * N, "launches": stats["count"]}
    if name:
        out["kernel"] = DOMINANT[name]["kernel"]
    if brief:
        return out
    kv = counter_summary(name) if (name and counted) else None
    out["traffic"] = (float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])
                      if kv else None)
    if kv and "valu_insts_per_launch" in kv:
        insts = float(kv["valu_insts_per_launch"])
        floor_ms = insts / (N_CU * CLOCK_GHZ * 1e9) * 1e3  # one wave-instruction/CU/cycle
        out["vector_issue"] = {
            "valu_wave_insts_per_launch": insts,
            "floor_ms_at_2.4GHz": floor_ms,
            "issue_frac": floor_ms / ms,
            "profiled_insts_per_cu_cycle": float(kv.get("valu_insts_per_cu_cycle", "nan")),
            "mix": kv.get("valu_mix", "")}
    if kv and "trace_mean_us" in kv:
        out["kernel_ms_rocprofv3"] = float(kv["trace_mean_us"]) * 1e-3
    if kv and "trace_isolated_mean_us" in kv:
        # the dispatches the event-timed call made (see read_trace_csv)
        out["kernel_ms_rocprofv3_event_call"] = float(kv["trace_isolated_mean_us"]) * 1e-3
    return out


def copy_bandwidth(torch) -> float:
    """GB/s of a 1 GiB device-to-device copy (read + write), events on the stream."""
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(2):
        b.copy_(a)
    stream = torch.cuda.current_stream()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for _ in range(10):
        b.copy_(a)
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / 10
    del a, b
    torch.cuda.empty_cache()
    return 2 * (1 << 30) / (ms * 1e-3) / 1e9


def fit_multi_hit(ms_by_k: dict, ms0: float, N: int) -> dict:
    """The paper's multi-hit law: per-hit time t(k) = t_inf + c / k, where c is the
    memory (load and store) cost of a site's Monte Carlo update and t_inf the cost of a
    hit.  t(k) is the Monte Carlo phase's time per hit, (sweep(k) - sweep(0)) / (N k)."""
    import numpy as np
    ks = sorted(k for k in ms_by_k if k > 0)
    t = np.array([(ms_by_k[k] - ms0) * 1e9 / (N * k) for k in ks])  # ps per hit
    A = np.stack([np.ones(len(ks)), 1.0 / np.array(ks, dtype=float)], axis=1)
    (t_inf, c), *_ = np.linalg.lstsq(A, t, rcond=None)
    fit = A @ np.array([t_inf, c])
    return {"k": ks, "t_ps_per_hit": t.tolist(), "fit_ps": fit.tolist(),
            "max_rel_residual": float(np.max(np.abs(fit - t) / t)),
            "t_inf_ps": float(t_inf), "c_ps": float(c),
            "hits_per_ns_asymptotic": 1e3 / float(t_inf),
            "ms_per_sweep_k0": ms0,
            "note": "t(k) = (sweep(k) - sweep(k=0)) / (N k), both with the same over-relaxation"}


def large_lattice_leg(hsg, torch, args) -> dict:
    """The largest lattice of the large-lattice configuration, L = 512 (134M spins),
    binary32 and binary64 (3.2 and 6.4 GB of spins and couplings), the headline sweep
    (k + n_or, T, renormalisation), the library's traversal for each precision."""
    L = 512
    N = L ** 3
    out = {}
    for dt, name, scale in ((torch.float32, "f32", 1), (torch.float64, "f64", 2)):
        lat = hsg.Lattice(L, dt, seed=1)
        flags = hsg.default_flags(L, dt)
        steps = max(4, args.steps // 5) if scale == 1 else 4
        ms = time_sweeps(lat, torch, T=args.T, k=args.k, n_or=args.n_or, R=args.renorm_every,
                         steps=steps, warmup=2, flags=flags)
        del lat
        torch.cuda.empty_cache()
        rec = {"L": L, "dtype": name, "k": args.k, "n_or": args.n_or, "steps": steps,
               "flags": flags, "ms_per_step": ms,
               "spin_updates_per_ns": N * (args.k + args.n_or) / (ms * 1e6)}
        # the same byte model in each precision: 36 B per site and phase in binary32, 72 B
        # in binary64
        rec[f"hbm_frac_{int(36 * scale)}B"] = (N * (1 + args.n_or) * BYTES_PER_SITE_PHASE * scale
                                              / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
        if scale == 1:
            out.update(rec)
        else:
            out["binary64"] = rec
    return out


def main():
    args = parse()
    if args.reduce_counters:
        reduce_counters(*args.reduce_counters)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the library has no multi-GPU path (asked for "
              f"--gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1006_2566_amd as hsg

    L, R = args.L, args.renorm_every
    N = L ** 3
    if args.flags is not None:
        flags = args.flags
    elif args.counters:
        # both dominant-kernel candidates are dispatched: Metropolis colour passes and
        # over-relaxation phases that carry the next colour-0 Metropolis pass
        flags = hsg.HSG_SNAKE | hsg.HSG_PHASE_MC
    elif args.no_autotune:
        flags = hsg.default_flags(L, torch.float32)
    else:
        from paper_1006_2566_amd import autotune
        flags = autotune.sweep_flags(L, torch.float32, k=args.k, n_or=args.n_or, T=args.T,
                                     renorm_every=args.renorm_every)
    lat = hsg.Lattice(L, torch.float32, seed=1)
    if args.counters:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)  # 1 GiB read + 1 GiB written
        torch.cuda.synchronize()
        # four sweeps (an even number of phase launches): three launches carrying the next
        # colour-0 Metropolis pass, one plain phase, five Metropolis colour passes
        lat.sweep(T=args.T, k=args.k, n_or=args.n_or, renorm_every=R, n_sweeps=4, flags=flags)
        torch.cuda.synchronize()
        return

    per_k = {}
    ks = [args.k] + [int(x) for x in args.also_k.split(",") if x.strip()]
    for k in ks:
        ms = time_sweeps(lat, torch, T=args.T, k=k, n_or=args.n_or, R=R, steps=args.steps,
                         warmup=args.warmup, flags=flags)
        upd = N * (k + args.n_or) / (ms * 1e6)
        per_k[str(k)] = {"ms_per_step": ms, "spin_updates_per_ns": upd,
                         "site_sweeps_per_ns": N / (ms * 1e6),
                         "hbm_frac_36B": N * (1 + args.n_or) * BYTES_PER_SITE_PHASE /
                         (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        note(f"k={k}: {upd:.1f} spin updates/ns (flags {flags})")

    # Every launch of the headline sweep timed with HIP events on the launch stream
    # (hsg_sweep_timed, the same sweeps): per-kind durations, the dominant kernel's
    # roofline against its algorithmic bytes (36 B per site-phase).
    launches = traced_launches(hsg, lat, T=args.T, k=args.k, n_or=args.n_or, R=R,
                               n=args.steps, flags=flags)
    dom_kind = max((kd for kd in launches if kd in LAUNCH_ROOFLINE),
                   key=lambda kd: launches[kd]["total_ms"])
    roofline = kernel_roofline(dom_kind, launches[dom_kind], N, counted=L == 256 and args.k == 4)
    roofline["launches"] = {hsg.LAUNCH_NAMES[kd]: v for kd, v in launches.items()}
    # the event-timed call's launches summed per sweep, against ms_per_step of the plain
    # call (the timed region): the per-launch durations account for the whole sweep
    roofline["launches_sum_ms_per_step"] = (sum(v["total_ms"] for v in launches.values())
                                            / args.steps)
    note(f"roofline: {roofline['kernel']} {roofline['kernel_ms'] * 1e3:.1f} us, "
         f"frac {roofline['frac']:.3f}")
    copy = copy_bandwidth(torch)
    roofline["copy_GBs"] = copy
    roofline["frac_of_copy"] = roofline["achieved"] / copy
    # the headline sweep against each byte model: fraction of the HBM peak and of the
    # measured copy bandwidth
    for kk, rec_k in per_k.items():
        gb_per_s = {m: N * (1 + args.n_or) * b / (rec_k["ms_per_step"] * 1e-3) / 1e9
                    for m, b in BYTE_MODELS.items()}
        rec_k["byte_models"] = {m: {"GBs": v, "frac_of_peak": v / HBM_PEAK_GBS,
                                    "frac_of_copy": v / copy} for m, v in gb_per_s.items()}
    # counter-measured bytes of one steady-state sweep of the default traversal (one
    # Metropolis colour pass + one phase launch carrying the next colour-0 pass)
    kv_mc, kv_ph = counter_summary("metropolis_pass"), counter_summary("phase_mc")
    if L == 256 and args.k == 4 and args.n_or == 1 and kv_mc and kv_ph and \
            dom_kind == 4:
        measured = sum(float(kv[f]) for kv in (kv_mc, kv_ph)
                       for f in ("fetch_bytes_per_launch", "write_bytes_per_launch"))
        roofline["sweep_bytes_measured"] = measured
        roofline["sweep_bytes_measured_vs_36B"] = measured / (N * (1 + args.n_or) *
                                                              BYTES_PER_SITE_PHASE)
    # the other kinds of launch of the headline sweep against the same roofline
    roofline["others"] = {hsg.LAUNCH_NAMES[kd]: kernel_roofline(kd, launches[kd], N, counted=False,
                                                                brief=True)
                          for kd in launches if kd in LAUNCH_ROOFLINE and kd != dom_kind}

    # the multi-hit law of the paper (§5, Table 3): per-hit time of the Monte Carlo phase,
    # t(k) = (sweep(k) - sweep(k=0)) / (N k), fitted to t_inf + c / k
    ms0 = time_sweeps(lat, torch, T=args.T, k=0, n_or=args.n_or, R=R, steps=args.steps,
                      warmup=2, flags=flags)
    multi_hit = fit_multi_hit({int(k): v["ms_per_step"] for k, v in per_k.items()}, ms0, N)
    note(f"multi-hit: t_inf {multi_hit['t_inf_ps']:.2f} ps/hit, c {multi_hit['c_ps']:.2f} ps")

    head = per_k[str(args.k)]
    rec = {"metric": METRIC,
           "value": head["spin_updates_per_ns"], "unit": "spin updates/ns", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"single lattice L={L} binary32, Gaussian couplings, "
                                  f"T={args.T}, sweep = Metropolis k={args.k} + "
                                  f"{args.n_or} over-relaxation, renormalise every {R}",
                      "L": L, "k": args.k, "n_or": args.n_or, "T": args.T, "flags": flags},
           "per_k": per_k, "roofline": roofline, "multi_hit": multi_hit}
    if args.large_L:
        rec["large_lattice"] = large_lattice_leg(hsg, torch, args)
        note("large-lattice leg done")
    if not args.no_binary64:
        rec["binary64"] = binary64_leg(hsg, args, torch, flags if args.flags is not None
                                       else hsg.default_flags(L, torch.float64))
        note("binary64 leg done")
    if not args.no_heat_bath:
        rec["heat_bath"] = heat_bath_leg(hsg, lat, torch, args, flags)
        note("heat-bath leg done")
    if args.large_L:  # with the other extra lattice sizes
        rec["paper_workload"] = paper_workload_leg(hsg, torch)
        note(f"paper workload: {rec['paper_workload']['ns_per_update'] * 1e3:.2f} ps per "
             f"update")
    if not args.no_observables:
        rec["observables"] = observables_leg(hsg, lat, torch, args.steps)
        note("observables leg done")
    if args.batch_cycles > 0:
        del lat
        torch.cuda.empty_cache()
        rec["batched"] = batched_leg(args, torch)
        note("batched leg done")
    if args.serve_requests > 0:
        torch.cuda.empty_cache()
        rec["served"] = served_leg(args, torch)
        note("served leg done")
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(args)
        note("cpu baseline done")
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
