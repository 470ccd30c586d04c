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
# 32-bit vector ALU peak of MI355X: the 157.3 TFLOP/s binary32 vector figure counts a
# fused multiply-add as 2 flops, so 78.6e12 lane operations per second (256 compute
# units x 128 lanes x 2.4 GHz).
ALU_PEAK_TOPS = 157.3 / 2
# Algorithmic 32-bit lane operations of the Metropolis pass (a fused multiply-add, a
# compare, a select, each half of a 32x32->64 product counts one):
#   per site:  local field 3 x (1 mul + 5 fma) = 18, sigma.h 3         -> 21
#   per Philox4x32-10 block: 10 rounds x (2 products x 2 halves + 4 xor) = 80;
#              a hit takes three of a block's four words, so k hits draw
#              ceil(3k / 4) blocks
#   per hit:   three uniforms 3 x (shift, or, convert, scale)           = 12
#              trial point: 2u-1, 1-z^2, sqrt, 4u, rint, r, r^2, sin (5), cos (5),
#              quadrant (convert, and, 4 selects), rho cos, rho sin     = 25
#              decision: s.h (3), dE, -beta dE, exp (2), dE <= 0, u < p, or,
#              4 selects (spin, s.h), energy sum (convert, add)         = 16
OPS_PER_SITE = 21
OPS_PER_BLOCK = 80
OPS_PER_HIT = 12 + 25 + 16
# over-relaxation of a site: local field and sigma.h (21), h.h (3), 2 sigma.h / h.h (2),
# h.h > 0 (1), reflection 3 x (fma, select) (6)
OPS_PER_SITE_OR = 21 + 3 + 2 + 1 + 6


def ops_per_site_pass(k: int) -> int:
    """Algorithmic lane operations of one site's Metropolis update with k hits."""
    return OPS_PER_SITE + OPS_PER_HIT * k + OPS_PER_BLOCK * ((3 * k + 3) // 4)


# Heat-bath draw (exact sample of exp(beta sigma.h) on the sphere), each library
# function (expm1, log1p or log, square root, division) counted as one operation:
#   two uniforms 2 x (shift-in, subtract)                                = 4
#   |h|: h.h (3), root, a = beta |h|, a > 0                              = 6
#   cosine to the field: 1 - u0, -2a, expm1, w q (2), w q <= 1/2,
#     log1p or log (3), divide, add, two clamps (4)                      = 15
#   rho = sqrt(1 - c^2) (2), azimuth as the Metropolis trial point (20) = 22
#   frame about h/|h|: h.h > 0, three divisions, sign (2), -1/(sgn + n_z)
#     (2), b (2), e1 (6), e2 (3)                                         = 19
#   point: rho cos, rho sin, three components x (mul, fma, fma)          = 11
#   energy change and sum: trial.h (3), dE, convert, add                = 6
# A draw takes two of a block's four words: k draws draw ceil(k / 2) blocks.
OPS_PER_DRAW = 4 + 6 + 15 + 22 + 19 + 11 + 6


def ops_per_site_heat_bath(k: int) -> int:
    """Algorithmic lane operations of one site's heat-bath update with k draws."""
    return OPS_PER_SITE + OPS_PER_DRAW * k + OPS_PER_BLOCK * ((k + 1) // 2)
_COMMON_SOURCES = ("paper_1006_2566_amd/csrc/hsg_site.h", "paper_1006_2566_amd/csrc/hsg_device.h",
                   "paper_1006_2566_amd/csrc/hsg_internal.h")
# The kernels that can dominate the headline sweep: the binary32 Metropolis colour pass,
# and the launch of the over-relaxation phase with the next sweep's colour-0 Metropolis
# pass (HSG_PHASE_MC).  Each has its counter summary, valid while its sources are those
# the counters were taken from.
DOMINANT = {
    "metropolis_pass": {
        "kernel": "colour_pass_kernel<float, Metropolis>",
        "trace_name": "colour_pass_kernel<float, (hsg::PassMode)0, false>",
        "sources": _COMMON_SOURCES + ("paper_1006_2566_amd/csrc/kernels_sweep.hip",),
        "traffic_file": "profiles/traffic_metropolis_pass_L256_f32.txt",
        "title": "one Metropolis colour pass",
        "sites": 0.5,  # updated sites per launch, in units of N
    },
    "phase_mc": {
        "kernel": "phase_kernel<float, 3, Metropolis>",
        "trace_name": "phase_kernel<float, 3, (hsg::PassMode)0>",
        "sources": _COMMON_SOURCES + ("paper_1006_2566_amd/csrc/kernels_phase.hip",),
        "traffic_file": "profiles/traffic_phase_mc_L256_f32.txt",
        "title": "one over-relaxation phase with the next colour-0 Metropolis pass",
        "sites": 1.0,  # the phase's compulsory traffic: every site read and written once
    },
}


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
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests of the served stream (0 skips that leg)")
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
    ap.add_argument("--no-observables", action="store_true",
                    help="skip timing the Fourier-overlap records (chi_SG, xi inputs)")
    ap.add_argument("--counters", action="store_true",
                    help="short run for hardware-counter collection: one 1 GiB device copy "
                         "(calibrates FETCH_SIZE / WRITE_SIZE), then 3 sweeps of the headline "
                         "configuration; prints no JSON")
    ap.add_argument("--reduce-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn the counter_collection.csv files of a FETCH_SIZE and a "
                         "WRITE_SIZE run of --counters into the per-launch traffic summaries "
                         "of the kernels the run dispatched ("
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


def read_counter_csv(path):
    """{kernel name: [value per dispatch]} of one counter from rocprofv3's CSV."""
    import csv
    out = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def reduce_counters(fetch_csv, write_csv):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of each dominant-kernel candidate the
    run dispatched, each scaled by what the same counter reads for the 1 GiB device copy
    of the --counters run."""
    fetch, write = read_counter_csv(fetch_csv), read_counter_csv(write_csv)

    def pick(d, key):
        names = [n for n in d if key(n)]
        if len(names) > 1:
            raise SystemExit(f"expected one kernel, found {names}")
        return d[names[0]] if names else None

    copy_f = pick(fetch, lambda n: "copy" in n.lower())
    copy_w = pick(write, lambda n: "copy" in n.lower())
    if copy_f is None or copy_w is None:
        raise SystemExit("no device copy in the counter runs")
    gib_kib = float(1 << 20)
    f_scale = gib_kib / max(copy_f)
    w_scale = gib_kib / max(copy_w)
    written = 0
    for name, d in DOMINANT.items():
        k_f = pick(fetch, lambda n: d["trace_name"] in n)
        k_w = pick(write, lambda n: d["trace_name"] in n)
        if k_f is None or k_w is None:
            continue
        f_b = sum(k_f) / len(k_f) * 1024 * f_scale
        w_b = sum(k_w) / len(k_w) * 1024 * w_scale
        lines = [
            f"# HBM traffic of {d['title']} ({d['kernel']}), L=256 binary32, k=4",
            "# commands: rocprofv3 --pmc FETCH_SIZE -d <dir> -o run --output-format csv -- "
            "python bench.py --counters   (then the same with WRITE_SIZE)",
            "#           python bench.py --reduce-counters <fetch csv> <write csv>",
            f"copy_fetch_kib={max(copy_f):.0f} fetch_scale={f_scale:.4f}",
            f"copy_write_kib={max(copy_w):.0f} write_scale={w_scale:.4f}",
            f"dispatches={len(k_f)}",
            f"fetch_bytes_per_launch={f_b:.0f}",
            f"write_bytes_per_launch={w_b:.0f}",
            f"algorithmic_bytes_per_launch={(1 << 24) * d['sites'] * BYTES_PER_SITE_PHASE:.0f}",
            f"source_hash={source_hash(name)}",
        ]
        with open(os.path.join(ROOT, d["traffic_file"]), "w") as f:
            f.write("\n".join(lines) + "\n")
        print("\n".join(lines))
        written += 1
    if not written:
        raise SystemExit("none of the dominant-kernel candidates was dispatched")


def measured_traffic(name: str):
    """Copy-calibrated HBM bytes per launch of a dominant-kernel candidate from its
    committed counter summary, or None when its sources changed since the counters were
    taken."""
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
    if kv.get("source_hash") != source_hash(name):
        return None
    return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])


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


def heat_bath_leg(hsg, lat, torch, args, flags, pass_flags):
    """The headline sweep with k heat-bath draws per site in place of the Metropolis
    hits (same traversal), and the heat-bath colour pass alone against the vector-ALU
    roofline (Metropolis-free sweeps, two passes each, events on the launch stream)."""
    N = lat.L ** 3
    steps = max(10, args.steps // 2)
    ms = time_sweeps(lat, torch, T=args.T, k=args.k, n_or=args.n_or, R=args.renorm_every,
                     steps=steps, warmup=2, flags=flags | hsg.HSG_HEAT_BATH)
    ms_pass = time_sweeps(lat, torch, T=args.T, k=args.k, n_or=0, R=0, steps=steps, warmup=2,
                          flags=pass_flags | hsg.HSG_HEAT_BATH) / 2.0
    ops = N / 2 * ops_per_site_heat_bath(args.k)
    tops = ops / (ms_pass * 1e-3) / 1e12
    return {"k_draws": args.k, "steps": steps, "ms_per_step": ms, "flags": flags | hsg.HSG_HEAT_BATH,
            "spin_updates_per_ns": N * (args.k + args.n_or) / (ms * 1e6),
            "pass": {"kernel": "colour_pass_kernel<float, HeatBath>", "bound": "alu",
                     "kernel_ms": ms_pass, "ops_per_launch": ops, "achieved": tops,
                     "peak": ALU_PEAK_TOPS, "unit": "TOP/s", "frac": tops / ALU_PEAK_TOPS,
                     "draws_per_ns": N / 2 * args.k / (ms_pass * 1e6)}}


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
    return {"workload": "256 samples x 2 replicas x 24 temperatures (12288 chains, "
                        f"{sites:.3g} spins), L in {{16,24,32,48}}, binary32, k=4, exchange "
                        "every 10 sweeps, overlap every 100, one graph per 100 sweeps",
            "sweeps": sweeps, "ms": ms, "ms_per_sweep": ms / sweeps,
            "spin_updates_per_ns": upd,
            "plain_per_lattice_updates_per_ns": upd_plain,
            "speedup_vs_plain": upd / upd_plain,
            "exchange_acceptance_per_pair_round": acc,
            "threads": b.threads}


def served_leg(args, torch):
    """Request stream: Poisson arrivals at 200 per second, L uniform in
    {8,16,32,64,96}, T uniform in [0.1,1], sweeps log-uniform in [100,10000], k in
    {1,4}, binary32, admitted by device-memory footprint, lattices resident between
    steps, continuous batching; latency = completion - arrival (wall clock)."""
    import numpy as np

    from paper_1006_2566_amd import serve as S

    trace = S.poisson_trace(n=args.serve_requests, rate=200.0, seed=1)
    tile = args.serve_tile or 256
    if not args.serve_tile and not args.no_autotune:
        from paper_1006_2566_amd import autotune
        tile = autotune.serve_shape(trace[:64])["tile_sites"]
    srv = S.Server(hbm_budget=args.serve_budget_mb << 20, n_slots=2048,
                   step_sweeps=args.serve_step, tile_sites=tile)
    srv.run([S.Request(rid=-1, seed=1, L=8, T=1.0, sweeps=2, k=1)], realtime=False)  # load kernels
    t0 = time.perf_counter()
    res = srv.run(trace, realtime=True)
    wall = time.perf_counter() - t0
    upd = float(sum(r.L ** 3 * r.sweeps * r.k for r in trace))
    offered = upd / trace[-1].arrival / 1e9
    st = S.latency_stats(res)
    # the same kind of requests through the plain per-lattice path, one after another
    # (initial state, sweeps with hsg_sweep, energy read back): the first 40 of the trace
    import paper_1006_2566_amd as hsg
    sample = trace[:40]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for r in sample:
        lat = hsg.Lattice(r.L, torch.float32, seed=r.seed)
        lat.sweep(T=r.T, k=r.k, n_or=0, n_sweeps=r.sweeps)
        lat.energy().item()
        del lat
    torch.cuda.synchronize()
    plain = sum(r.L ** 3 * r.sweeps * r.k for r in sample) / ((time.perf_counter() - t1) * 1e9)
    return {"workload": f"{len(trace)} requests, Poisson 200/s, L in {{8,16,32,64,96}}, "
                        "T in [0.1,1], sweeps log-uniform [100,1e4], k in {1,4}, binary32",
            "p50_latency_s": st["p50_s"], "p99_latency_s": st["p99_s"],
            "mean_latency_s": st["mean_s"], "wall_s": wall,
            "spin_updates_per_ns": upd / (wall * 1e9),
            "offered_updates_per_ns": offered,
            "plain_per_lattice_updates_per_ns": plain,
            "speedup_vs_plain": upd / (wall * 1e9) / plain, "budget_mb": args.serve_budget_mb,
            "step_sweeps": args.serve_step, "tile_sites": tile,
            "scheduler": {k: (round(v, 3) if isinstance(v, float) else v)
                          for k, v in srv.stats.items()}}


def cpu_baseline(args):
    """The CPU oracle, unchanged, on the host cores: the same L, k, n_or and T,
    as many whole sweeps as fit in about args.cpu_seconds (at least one)."""
    import numpy as np

    import oracle as O

    L = args.L
    spins, J = O.init(L, 1, np.float32)
    E = O.energy(L, spins, J)
    n = 0
    t0 = time.perf_counter()
    while True:
        r = O.sweep(L, 1, spins, J, T=args.T, k=args.k, n_or=args.n_or,
                    renorm_every=args.renorm_every, n_sweeps=1, sweep0=n, E=E)
        E = r["E"]
        n += 1
        if time.perf_counter() - t0 >= args.cpu_seconds:
            break
    dt = time.perf_counter() - t0
    updates = L ** 3 * (args.k + args.n_or) * n
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": updates / (dt * 1e9), "unit": "spin updates/ns", "cores": cores,
            "kind": "oracle",
            "sample": f"L={L} binary32, {n} sweep(s) of k={args.k} Metropolis + {args.n_or} "
                      f"over-relaxation, T={args.T}, {dt:.1f} s wall"}


def main():
    args = parse()
    if args.reduce_counters:
        reduce_counters(*args.reduce_counters)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for "
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
        lat.sweep(T=args.T, k=args.k, n_or=args.n_or, renorm_every=R, n_sweeps=3, flags=flags)
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

    # The Metropolis colour pass (half the sites, k hits each): its average duration from
    # Metropolis-only sweeps (two passes each, one energy fold per call) timed with events
    # on the launch stream.  The over-relaxation pass, bound by HBM, is timed the same way.
    pass_flags = flags & ~(hsg.HSG_FUSED | hsg.HSG_PHASE_LAUNCH | hsg.HSG_PHASE_MC)
    ms_mh_pass = time_sweeps(lat, torch, T=args.T, k=args.k, n_or=0, R=0, steps=args.steps,
                             warmup=2, flags=pass_flags) / 2.0
    ms_or_pass = time_sweeps(lat, torch, T=args.T, k=0, n_or=1, R=0, steps=args.steps,
                             warmup=2, flags=pass_flags) / 2.0
    # the over-relaxation phase as one launch (when the traversal uses it): both passes
    # of the phase, 36 B per site algorithmic
    or_phase = None
    phase = bool(flags & (hsg.HSG_PHASE_LAUNCH | hsg.HSG_PHASE_MC)) and hsg.phase_supported(L)
    if phase:
        ms_ph = time_sweeps(lat, torch, T=args.T, k=0, n_or=1, R=0, steps=args.steps, warmup=2,
                            flags=flags)
        gbs = N * BYTES_PER_SITE_PHASE / (ms_ph * 1e-3) / 1e9
        or_phase = {"kernel": "phase_kernel<float, 2, OverRelax>", "bound": "hbm",
                    "kernel_ms": ms_ph, "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}
    head = per_k[str(args.k)]
    sites_pass = N / 2
    ops_pass = sites_pass * ops_per_site_pass(args.k)
    achieved = ops_pass / (ms_mh_pass * 1e-3) / 1e12
    counted = L == 256 and args.k == 4
    metropolis = {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS, "unit": "TOP/s",
                  "frac": achieved / ALU_PEAK_TOPS,
                  "traffic": measured_traffic("metropolis_pass") if counted else None,
                  "kernel": DOMINANT["metropolis_pass"]["kernel"], "kernel_ms": ms_mh_pass,
                  "ops_per_launch": ops_pass,
                  "hits_per_ns": sites_pass * args.k / (ms_mh_pass * 1e6),
                  "hbm_frac_36B": sites_pass * BYTES_PER_SITE_PHASE / (ms_mh_pass * 1e-3) /
                  1e9 / HBM_PEAK_GBS}
    extras = {"overrelax_pass": {"bound": "hbm", "kernel_ms": ms_or_pass,
                                 "achieved_GBs": sites_pass * BYTES_PER_SITE_PHASE /
                                 (ms_or_pass * 1e-3) / 1e9,
                                 "frac": sites_pass * BYTES_PER_SITE_PHASE /
                                 (ms_or_pass * 1e-3) / 1e9 / HBM_PEAK_GBS},
              "overrelax_phase": or_phase}
    if phase and flags & hsg.HSG_PHASE_MC and args.k > 0 and args.n_or > 0:
        # Dominant kernel: the over-relaxation phase with the next sweep's colour-0
        # Metropolis pass.  A call of n sweeps runs n + 1 Metropolis passes, n - 1 such
        # launches, (n - 1)(n_or - 1) + n_or plain phases and fixed per-call work, so the
        # growth of the call's time per sweep (two call lengths, events on the launch
        # stream) less a Metropolis pass and n_or - 1 phases is the launch's duration.
        n1, n2 = max(4, args.steps // 5), max(args.steps, 2 * max(4, args.steps // 5))
        tot = [time_sweeps(lat, torch, T=args.T, k=args.k, n_or=args.n_or, R=0, steps=n,
                           warmup=2, flags=flags) * n for n in (n1, n2)]
        ms_f = (tot[1] - tot[0]) / (n2 - n1) - ms_mh_pass - (args.n_or - 1) * or_phase["kernel_ms"]
        bytes_f = N * BYTES_PER_SITE_PHASE
        ops_f = sites_pass * ops_per_site_pass(args.k) + N * OPS_PER_SITE_OR
        gbs_f = bytes_f / (ms_f * 1e-3) / 1e9
        tops_f = ops_f / (ms_f * 1e-3) / 1e12
        # the larger of the two floors binds: the phase's compulsory bytes at HBM peak
        # against both passes' lane operations at the vector peak
        hbm_bound = bytes_f / HBM_PEAK_GBS >= ops_f / (ALU_PEAK_TOPS * 1e3)
        roofline = {"bound": "hbm" if hbm_bound else "alu",
                    "achieved": gbs_f if hbm_bound else tops_f,
                    "peak": HBM_PEAK_GBS if hbm_bound else ALU_PEAK_TOPS,
                    "unit": "GB/s" if hbm_bound else "TOP/s",
                    "frac": gbs_f / HBM_PEAK_GBS if hbm_bound else tops_f / ALU_PEAK_TOPS,
                    "traffic": measured_traffic("phase_mc") if counted else None,
                    "kernel": DOMINANT["phase_mc"]["kernel"], "kernel_ms": ms_f,
                    "bytes_per_launch": bytes_f, "ops_per_launch": ops_f,
                    "alu_achieved": tops_f, "alu_frac": tops_f / ALU_PEAK_TOPS,
                    "metropolis_pass": metropolis, **extras}
    else:
        roofline = {**metropolis, **extras}

    rec = {"metric": METRIC,
           "value": head["spin_updates_per_ns"], "unit": "spin updates/ns", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"single lattice L={L} binary32, Gaussian couplings, "
                                  f"T={args.T}, sweep = Metropolis k={args.k} + "
                                  f"{args.n_or} over-relaxation, renormalise every {R}",
                      "L": L, "k": args.k, "n_or": args.n_or, "T": args.T, "flags": flags},
           "per_k": per_k, "roofline": roofline}
    note(f"roofline: {roofline['kernel']} {roofline['kernel_ms'] * 1e3:.1f} us, "
         f"frac {roofline['frac']:.3f}")
    if not args.no_binary64:
        rec["binary64"] = binary64_leg(hsg, args, torch, flags if args.flags is not None
                                       else hsg.default_flags(L, torch.float64))
        note("binary64 leg done")
    if not args.no_heat_bath:
        rec["heat_bath"] = heat_bath_leg(hsg, lat, torch, args, flags, pass_flags)
        note("heat-bath leg done")
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
