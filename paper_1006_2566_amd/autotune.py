"""Autotuner: launch shapes and traversal orders chosen by timing them on the device.

Every choice here only changes how the work is laid out on the GPU -- the traversal
order of the colour passes, the workgroup size of the batched sweep, the tile size and
step length of the served passes -- never a spin or a decision (the GPU tests check
that each candidate reproduces the others bit for bit).  The fastest candidate for a
workload is cached in a JSON file keyed by the device architecture and the workload, so
tuning runs once per machine.

Cache file: ``$HSG_AUTOTUNE_CACHE`` if set, else
``~/.cache/paper_1006_2566_amd/autotune.json``.
"""
from __future__ import annotations

import json
import os
import time
from typing import Callable, Iterable

import torch

from . import (HSG_FUSED, HSG_PHASE_LAUNCH, HSG_PHASE_MC, HSG_SNAKE, Lattice, fused_supported,
               phase_supported)

CACHE_ENV = "HSG_AUTOTUNE_CACHE"


def cache_path() -> str:
    return os.environ.get(CACHE_ENV) or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1006_2566_amd", "autotune.json")


def device_key() -> str:
    """Architecture of the current device, e.g. 'gfx950:sramecc+:xnack-'."""
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(props, "gcnArchName", props.name)


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(data: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def pick(key: str, candidates: Iterable, measure: Callable[[object], float], *,
         retune: bool = False, path: str | None = None, dev: str | None = None):
    """The cached winner for `key`, else the candidate with the smallest measure(c)
    (milliseconds), which is then cached.  Candidates must be JSON-serialisable."""
    cands = list(candidates)
    if not cands:
        raise ValueError("no candidates")
    dev = dev or device_key()
    cache = load_cache(path)
    entry = cache.get(dev, {}).get(key)
    if entry is not None and not retune and entry.get("choice") in cands:
        return entry["choice"]
    times = {json.dumps(c): float(measure(c)) for c in cands}
    best = min(cands, key=lambda c: times[json.dumps(c)])
    cache = load_cache(path)  # re-read: another process may have tuned meanwhile
    cache.setdefault(dev, {})[key] = {"choice": best, "ms": times, "when": time.time()}
    save_cache(cache, path)
    return best


def _event_ms(fn: Callable[[], None], reps: int) -> float:
    stream = torch.cuda.current_stream()
    fn()  # warm-up (first launches, caches)
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(reps):
        fn()
    t1.record(stream)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / reps


def sweep_flags(L: int, dtype: torch.dtype = torch.float32, k: int = 4, n_or: int = 1,
                heat_bath: bool = False, T: float = 0.3, renorm_every: int = 10,
                retune: bool = False, path: str | None = None) -> int:
    """Traversal flags for hsg_sweep on an L^3 lattice: plain order, alternating z
    order (HSG_SNAKE), over-relaxation phases in one launch each (HSG_PHASE_LAUNCH), the
    same with the next sweep's colour-0 Monte Carlo pass in that launch (HSG_PHASE_MC) or
    fused passes (HSG_FUSED), where the lattice allows them."""
    cands = [0, HSG_SNAKE]
    if n_or > 0 and phase_supported(L):
        cands.append(HSG_SNAKE | HSG_PHASE_LAUNCH)
        if k > 0:
            cands.append(HSG_SNAKE | HSG_PHASE_MC)
    if fused_supported(L):
        cands.append(HSG_FUSED)
    key = f"sweep L={L} {str(dtype).replace('torch.', '')} k={k} n_or={n_or} hb={int(heat_bath)}"
    best: dict = {}

    def measure(flags):
        # All candidates are timed on one lattice (flags never change a spin), in turn
        # over three rounds, and each keeps its fastest round: a clock that drifts
        # during tuning then favours none of them.
        if not best:
            lat = Lattice(L, dtype, seed=1)
            for _ in range(3):
                for c in cands:
                    ms = _event_ms(lambda: lat.sweep(T=T, k=k, n_or=n_or,
                                                     renorm_every=renorm_every, n_sweeps=8,
                                                     heat_bath=heat_bath, flags=c), 2)
                    best[c] = min(best.get(c, ms), ms)
            del lat
        return best[flags]
    return int(pick(key, cands, measure, retune=retune, path=path))


def batch_threads(batch, n_sweeps: int = 1, retune: bool = False,
                  path: str | None = None) -> int:
    """Workgroup size of hsg_batch_sweep for this batch (chain sizes, k, n_or)."""
    from collections import Counter
    hist = sorted(Counter((int(c.L), int(c.k), int(c.n_or)) for c in batch.specs).items())
    key = f"batch {str(batch.dtype).replace('torch.', '')} {hist}"
    saved = (batch.threads, batch.sweep_ctr.clone(), batch.E.clone(), batch.spins.clone(),
             batch.remaining.clone() if batch.remaining is not None else None)

    def measure(threads):
        batch.threads = threads
        return _event_ms(lambda: batch.sweep(n_sweeps), 2)
    best = int(pick(key, [64, 128, 256, 512, 1024], measure, retune=retune, path=path))
    # the timing sweeps advanced the chains: put the batch back as it was
    batch.threads = best
    batch.sweep_ctr.copy_(saved[1])
    batch.E.copy_(saved[2])
    batch.spins.copy_(saved[3])
    if saved[4] is not None:
        batch.remaining.copy_(saved[4])
    return best


def serve_shape(trace_sample, budget_mb: int = 1024, retune: bool = False,
                path: str | None = None) -> dict:
    """Tile size of the served multi-lattice passes, timed on a closed batch of
    requests (all admitted at once): {"tile_sites": n}."""
    from . import serve as S
    key = f"serve tiles {sorted(set((r.L, r.k) for r in trace_sample))}"

    def measure(tile):
        srv = S.Server(hbm_budget=budget_mb << 20, n_slots=max(8, 2 * len(trace_sample)),
                       tile_sites=tile, step_sweeps=8)
        reqs = [S.Request(rid=i, seed=r.seed, L=r.L, T=r.T, sweeps=16, k=r.k)
                for i, r in enumerate(trace_sample)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        srv.run(reqs, realtime=False)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3
    tile = int(pick(key, [128, 256, 512, 1024], measure, retune=retune, path=path))
    return {"tile_sites": tile}
