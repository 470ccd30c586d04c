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

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
BYTES_PER_SITE_PHASE = 36.0  # binary32: read spin (12) + 3 bonds (12), write spin (12)


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
    ap.add_argument("--batch-threads", type=int, default=256)
    ap.add_argument("--serve-requests", type=int, default=1000,
                    help="requests of the served stream (0 skips that leg)")
    ap.add_argument("--serve-budget-mb", type=int, default=8192,
                    help="device memory for resident lattices of the served stream")
    ap.add_argument("--serve-step", type=int, default=16, help="sweeps per scheduling step")
    ap.add_argument("--counters", action="store_true",
                    help="short run for hardware-counter collection: one 1 GiB device copy "
                         "(calibrates FETCH_SIZE / WRITE_SIZE), then 2 sweeps of the headline "
                         "configuration; prints no JSON")
    return ap.parse_args()


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
    b = B.Batch(specs, threads=args.batch_threads)
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
            "threads": args.batch_threads}


def served_leg(args, torch):
    """Request stream: Poisson arrivals at 200 per second, L uniform in
    {8,16,32,64,96}, T uniform in [0.1,1], sweeps log-uniform in [100,10000], k in
    {1,4}, binary32, admitted by device-memory footprint, lattices resident between
    steps, continuous batching; latency = completion - arrival (wall clock)."""
    import numpy as np

    from paper_1006_2566_amd import serve as S

    trace = S.poisson_trace(n=args.serve_requests, rate=200.0, seed=1)
    srv = S.Server(hbm_budget=args.serve_budget_mb << 20, n_slots=2048,
                   step_sweeps=args.serve_step)
    srv.run([S.Request(rid=-1, seed=1, L=8, T=1.0, sweeps=2, k=1)], realtime=False)  # load kernels
    t0 = time.perf_counter()
    res = srv.run(trace, realtime=True)
    wall = time.perf_counter() - t0
    upd = float(sum(r.L ** 3 * r.sweeps * r.k for r in trace))
    offered = upd / trace[-1].arrival / 1e9
    st = S.latency_stats(res)
    return {"workload": f"{len(trace)} requests, Poisson 200/s, L in {{8,16,32,64,96}}, "
                        "T in [0.1,1], sweeps log-uniform [100,1e4], k in {1,4}, binary32",
            "p50_latency_s": st["p50_s"], "p99_latency_s": st["p99_s"],
            "mean_latency_s": st["mean_s"], "wall_s": wall,
            "spin_updates_per_ns": upd / (wall * 1e9),
            "offered_updates_per_ns": offered, "budget_mb": args.serve_budget_mb,
            "step_sweeps": args.serve_step,
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
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: this build has no multi-GPU path (asked for "
              f"--gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1006_2566_amd as hsg

    L, R = args.L, args.renorm_every
    N = L ** 3
    flags = hsg.DEFAULT_SWEEP_FLAGS if args.flags is None else args.flags
    lat = hsg.Lattice(L, torch.float32, seed=1)
    if args.counters:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)  # 1 GiB read + 1 GiB written
        torch.cuda.synchronize()
        lat.sweep(T=args.T, k=args.k, n_or=args.n_or, renorm_every=R, n_sweeps=2, flags=flags)
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

    # dominant kernel: the Metropolis colour pass.  Average duration of one such pass,
    # timed alone (k hits, no over-relaxation) with events on the launch stream.
    ms_mh_sweep = time_sweeps(lat, torch, T=args.T, k=args.k, n_or=0, R=0, steps=args.steps,
                              warmup=2, flags=flags)
    ms_pass = ms_mh_sweep / 2.0
    head = per_k[str(args.k)]
    bytes_pass = N / 2 * BYTES_PER_SITE_PHASE * 2 / 2  # 36 B per site-phase, half the sites
    roofline = {"bound": "hbm", "achieved": bytes_pass / (ms_pass * 1e-3) / 1e9,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": bytes_pass / (ms_pass * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                "kernel": "colour_pass_kernel<float, Metropolis>",
                "kernel_ms": ms_pass}

    rec = {"metric": "spin updates/ns at L=256 FP32 (k=1,4,8) + %HBM roofline",
           "value": head["spin_updates_per_ns"], "unit": "spin updates/ns", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"single lattice L={L} binary32, Gaussian couplings, "
                                  f"T={args.T}, sweep = Metropolis k={args.k} + "
                                  f"{args.n_or} over-relaxation, renormalise every {R}",
                      "L": L, "k": args.k, "n_or": args.n_or, "T": args.T, "flags": flags},
           "per_k": per_k, "roofline": roofline}
    if args.batch_cycles > 0:
        del lat
        torch.cuda.empty_cache()
        rec["batched"] = batched_leg(args, torch)
    if args.serve_requests > 0:
        torch.cuda.empty_cache()
        rec["served"] = served_leg(args, torch)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
