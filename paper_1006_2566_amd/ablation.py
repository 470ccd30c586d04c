"""The paper's kernel-design comparison (§4, Tables 2 and 3) re-run on this GPU.

The paper times five designs of the colour pass on its GPUs: GM (one launch per colour
pass over global memory), TEXT (GM with the read-only data fetched through the
texture path), CA (launches plane by plane so that a plane's neighbours stay in the
L1 cache), SM (three planes staged in shared memory, a z march) and SM4P (four planes,
two passes in flight), for the over-relaxation update at L = 128, and the multi-hit
cost of SM4P against the number of hits.  Here every design has an analogue selected by
sweep flags, and every analogue computes exactly the default schedule's spins:

    GM    0                                  one launch per colour pass
    GM+S  HSG_SNAKE                          GM, successive passes walking z backwards
    TEXT  HSG_SNAKE | HSG_STREAM_LOADS       read-only data with the non-temporal hint
    CA    HSG_PLANE_LAUNCH                   one launch per z plane (2L per phase)
    SM    HSG_FUSED | HSG_MARCH_PHASE        LDS plane march, one phase (2 passes) per launch
    SM4P  HSG_FUSED                          LDS plane march, up to four passes per launch
    PH    HSG_SNAKE | HSG_PHASE_LAUNCH       each over-relaxation phase as one launch (a
                                             lean one-phase LDS march; Metropolis phases
                                             pass by pass as in GM+S)
    PH+MC HSG_SNAKE | HSG_PHASE_MC           PH, the launch of each phase also running the
                                             next sweep's colour-0 Metropolis pass

The march needs 256 <= L <= 1024 (L a multiple of 64); elsewhere SM and SM4P are
reported as unsupported.  Workloads: over-relaxation only (the paper's Table 2) and
Metropolis with k hits plus one over-relaxation phase (the multi-hit question of Table
3).  Times are HIP events around `sweeps` sweeps after a warm-up; T_upd is ns per spin
update (N (k + n_or) updates per sweep), the paper's unit.

    python -m paper_1006_2566_amd.ablation [--L 256] [--sweeps 20] [--ks 0,1,4,8]
"""
from __future__ import annotations

import argparse
import json

import torch

from . import (HSG_FUSED, HSG_MARCH_PHASE, HSG_PHASE_LAUNCH, HSG_PHASE_MC, HSG_PLANE_LAUNCH,
               HSG_SNAKE, HSG_STREAM_LOADS, Lattice, fused_supported)

VARIANTS = {
    "GM": 0,
    "GM+S": HSG_SNAKE,
    "TEXT": HSG_SNAKE | HSG_STREAM_LOADS,
    "CA": HSG_PLANE_LAUNCH,
    "SM": HSG_FUSED | HSG_MARCH_PHASE,
    "SM4P": HSG_FUSED,
    "PH": HSG_SNAKE | HSG_PHASE_LAUNCH,
    "PH+MC": HSG_SNAKE | HSG_PHASE_MC,
}


def time_variant(L: int, flags: int, *, k: int, n_or: int, T: float, sweeps: int,
                 warmup: int, seed: int = 1):
    """(ms per sweep, final spins) of `warmup + sweeps` sweeps from the Philox state."""
    lat = Lattice(L, torch.float32, seed=seed)
    lat.sweep(T=T, k=k, n_or=n_or, renorm_every=10, n_sweeps=warmup, flags=flags)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    lat.sweep(T=T, k=k, n_or=n_or, renorm_every=10, n_sweeps=sweeps, flags=flags)
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / sweeps, lat.spins.clone(), float(lat.energy().item())


def run(L: int = 256, ks=(0, 1, 4, 8), sweeps: int = 20, warmup: int = 3, T: float = 0.3):
    """One row per (workload, variant): ms per sweep, T_upd, speed relative to GM, and
    whether the spins equal GM's bit for bit."""
    N = L ** 3
    rows = []
    for k in ks:
        n_or = 1
        ref = None
        for name, flags in VARIANTS.items():
            if flags & HSG_FUSED and not fused_supported(L):
                rows.append({"L": L, "k": k, "n_or": n_or, "variant": name, "flags": flags,
                             "supported": False})
                continue
            ms, spins, E = time_variant(L, flags, k=k, n_or=n_or, T=T, sweeps=sweeps,
                                        warmup=warmup)
            updates = N * (k + n_or)
            row = {"L": L, "k": k, "n_or": n_or, "variant": name, "flags": flags,
                   "supported": True, "ms_per_sweep": ms, "T_upd_ns": ms * 1e6 / updates,
                   "updates_per_ns": updates / (ms * 1e6), "E": E}
            if ref is None:
                ref = (ms, spins, E)
                row["same_spins_as_GM"] = True
            else:
                row["same_spins_as_GM"] = bool(torch.equal(spins, ref[1]))
            row["speed_vs_GM"] = ref[0] / ms
            rows.append(row)
            print(json.dumps(row), flush=True)
            del spins
        torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, default=256)
    ap.add_argument("--ks", default="0,1,4,8", help="Metropolis hits per sweep (0 = OR only)")
    ap.add_argument("--sweeps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--T", type=float, default=0.3)
    args = ap.parse_args()
    run(args.L, [int(x) for x in args.ks.split(",")], args.sweeps, args.warmup, args.T)


if __name__ == "__main__":
    main()
