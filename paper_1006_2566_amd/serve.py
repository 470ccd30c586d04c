"""Served form: continuous batching of simulation requests.

Requests (seed, L, T, sweeps, k) arrive over time.  The server admits them as
device memory and slots free up (admission by HBM footprint), keeps every admitted
lattice resident on the device, and advances all of them together in steps of a few
sweeps with ``hsg_batch_pass_sweep`` -- one launch per colour pass covering tiles of
every resident lattice, so requests that arrive while others run share the same
launches.  A request retires when its sweeps are done; its final energy and
magnetisation are read back and its memory is reused.

The loop is pipelined: each step is enqueued before the host looks at the previous
one, and every host<->device transfer goes through pinned memory without blocking,
so admission, tile building and retirement of step n overlap the GPU's work on step
n + 1 (the device never waits for the scheduler while lattices are resident).

Host-side scheduling only: every sweep, energy and magnetisation is computed by
libhsg's kernels.
"""
from __future__ import annotations

import bisect
import ctypes
import dataclasses
import math
import threading
import time
from collections import deque

import numpy as np
import torch

from . import _dtype_code, _ptr, _stream, check, lib
from .batch import BATCH_L_MAX, CHAIN_DTYPE, HSG_CHAIN_INIT_J, _Batch, _bind

DUMMY_L = 2  # placeholder lattice of a free slot (never swept: its budget is 0)


@dataclasses.dataclass
class Request:
    rid: int
    seed: int
    L: int
    T: float
    sweeps: int
    k: int
    arrival: float = 0.0  # seconds after the start of the run

    @property
    def spins(self) -> int:
        return self.L ** 3


@dataclasses.dataclass
class Result:
    rid: int
    E: float          # tracked energy after the last sweep (binary64)
    m: np.ndarray     # magnetisation (1/N) sum sigma_i, binary64
    arrival: float
    admitted: float
    finished: float
    admitted_step: int = -1  # scheduler iteration of admission
    finished_step: int = -1  # scheduler iteration that saw the lattice finished
    # "ok"; "cancelled" (E and m of the sweeps done, NaN if none were admitted);
    # "rejected: <reason>" (never admitted, E and m NaN)
    status: str = "ok"
    sweeps_done: int = -1  # sweeps the lattice made (-1: never admitted)

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def request_problem(req: Request, capacity_elements: int) -> str | None:
    """Why a request cannot be served (None if it can): L even in [2, BATCH_L_MAX], at
    least one Metropolis hit, T > 0 (T = inf means beta = 0), sweeps >= 0, a 64-bit
    seed, and a lattice whose 3 L^3 elements fit the spin (and coupling) arena."""
    if not (isinstance(req.L, int) and 2 <= req.L <= BATCH_L_MAX and req.L % 2 == 0):
        return f"L={req.L} must be even in [2, {BATCH_L_MAX}]"
    if not (1 <= req.k <= 0xFFFF):
        return f"k={req.k} must be in [1, 65535]"
    if not (req.T > 0):
        return f"T={req.T} must be > 0"
    if req.sweeps < 0 or req.sweeps > 0x7FFFFFFF:
        return f"sweeps={req.sweeps} out of range"
    if not (0 <= req.seed < 2 ** 64):
        return f"seed={req.seed} must fit 64 bits"
    if -(-3 * req.L ** 3 // 64) * 64 > capacity_elements:  # the arena's 64-element blocks
        return f"footprint of L={req.L} exceeds the device-memory budget"
    return None


def poisson_trace(n: int = 2000, rate: float = 200.0, seed: int = 1,
                  Ls=(8, 16, 32, 64, 96), T_range=(0.1, 1.0), sweep_range=(100, 10000),
                  ks=(1, 4)) -> list[Request]:
    """Synthetic request stream: Poisson arrivals at `rate` per second; request r has
    seed 1000 + r, L uniform in Ls, T uniform in T_range, sweeps log-uniform in
    sweep_range (rounded to an integer), k uniform in ks.  numpy PCG64 on `seed`."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n))
    Ls_ = rng.choice(np.asarray(Ls), size=n)
    Ts = rng.uniform(T_range[0], T_range[1], size=n)
    lo, hi = math.log(sweep_range[0]), math.log(sweep_range[1])
    sweeps = np.rint(np.exp(rng.uniform(lo, hi, size=n))).astype(np.int64)
    ks_ = rng.choice(np.asarray(ks), size=n)
    return [Request(rid=r, seed=1000 + r, L=int(Ls_[r]), T=float(Ts[r]), sweeps=int(sweeps[r]),
                    k=int(ks_[r]), arrival=float(arrivals[r])) for r in range(n)]


class Arena:
    """First-fit allocator over a range of elements (offsets into a device buffer)."""

    def __init__(self, size: int, align: int = 64):
        self.size, self.align = size, align
        self.free = [(0, size)]  # sorted, non-adjacent (start, end)

    def alloc(self, n: int) -> int | None:
        n = -(-n // self.align) * self.align
        for i, (a, b) in enumerate(self.free):
            if b - a >= n:
                if b - a == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (a + n, b)
                return a
        return None

    def release(self, start: int, n: int) -> None:
        n = -(-n // self.align) * self.align
        i = bisect.bisect_left(self.free, (start, start + n))
        self.free.insert(i, (start, start + n))
        merged = []
        for a, b in self.free:
            if merged and merged[-1][1] == a:
                merged[-1] = (merged[-1][0], b)
            else:
                merged.append((a, b))
        self.free = merged

    @property
    def used(self) -> int:
        return self.size - sum(b - a for a, b in self.free)


class PinnedRing:
    """Pinned host staging buffers reused in turn, each guarded by the event of the last
    copy that used it.  Allocating pinned memory while the GPU works can stall the host
    until the device is idle, so the server allocates all of it up front."""

    def __init__(self, n_buffers: int, nbytes: int):
        self.bufs = [torch.empty(nbytes, dtype=torch.uint8).pin_memory() for _ in range(n_buffers)]
        self.events: list[torch.cuda.Event | None] = [None] * n_buffers
        self.nbytes = nbytes
        self.i = 0

    def take(self) -> tuple[torch.Tensor, int]:
        """The next buffer (waiting for its previous copy if that is still running)."""
        k = self.i
        self.i = (self.i + 1) % len(self.bufs)
        if self.events[k] is not None:
            self.events[k].synchronize()
            self.events[k] = None
        return self.bufs[k], k

    def guard(self, k: int) -> None:
        """Record on the current stream that buffer k is in use up to this point."""
        ev = torch.cuda.Event()
        ev.record()
        self.events[k] = ev


class Server:
    """Continuous-batching server on one GPU.

    hbm_budget: bytes of device memory for resident lattices (spins + couplings);
    admission waits while a request's footprint does not fit.  n_slots bounds the
    number of resident lattices.  step_sweeps: sweeps per scheduling step."""

    def __init__(self, hbm_budget: int = 4 << 30, n_slots: int = 1024, step_sweeps: int = 16,
                 tile_sites: int = 256, dtype: torch.dtype = torch.float32,
                 device: str | torch.device = "cuda"):
        _bind()
        self.dtype, self.device = dtype, torch.device(device)
        self.es = torch.tensor([], dtype=dtype).element_size()
        self.step_sweeps, self.tile_sites = step_sweeps, tile_sites
        self.n_slots = n_slots
        # each lattice takes 3 L^3 spin elements and as many coupling elements
        per_buffer = hbm_budget // (2 * self.es)
        dummy = 3 * DUMMY_L ** 3
        self.dummy_base = per_buffer
        self.spins = torch.zeros(per_buffer + n_slots * dummy, dtype=dtype, device=self.device)
        self.J = torch.zeros(per_buffer + n_slots * dummy, dtype=dtype, device=self.device)
        self.arena_s = Arena(per_buffer)
        self.arena_j = Arena(per_buffer)
        # host staging: uploads (chain table, per-admission arrays) and read-backs
        self._h2d = PinnedRing(64, max(n_slots * CHAIN_DTYPE.itemsize, 16 * n_slots + 64))
        self._d2h = PinnedRing(8, 40 * n_slots + 64)
        self._tile_ring: PinnedRing | None = None
        self.table = np.zeros(n_slots, dtype=CHAIN_DTYPE)
        for s in range(n_slots):
            self._set_dummy(s)
        dev = self.device
        self.beta = torch.zeros(n_slots, dtype=torch.float64, device=dev)
        self.E = torch.zeros(n_slots, dtype=torch.float64, device=dev)
        self.sweep_ctr = torch.zeros(n_slots, dtype=torch.int32, device=dev)
        self.remaining = torch.zeros(n_slots, dtype=torch.int32, device=dev)
        self.order = torch.arange(n_slots, dtype=torch.int32, device=dev)
        self.chains = torch.empty(n_slots * CHAIN_DTYPE.itemsize, dtype=torch.uint8, device=dev)
        self._upload_table()
        self._d = _Batch(n_slots, _dtype_code(dtype), self.chains.data_ptr(),
                         self.spins.data_ptr(), self.J.data_ptr(), self.beta.data_ptr(),
                         self.E.data_ptr(), self.sweep_ctr.data_ptr(),
                         self.remaining.data_ptr(), self.order.data_ptr(), 256, 0)
        self.free_slots = list(range(n_slots - 1, -1, -1))
        # slot -> (request, spin offset, coupling offset, admission time, admission iteration)
        self.active: dict[int, tuple[Request, int, int, float, int]] = {}
        self._it = 0  # scheduler iteration of run()
        self._cancel_lock = threading.Lock()
        self._cancel_ids: set[int] = set()  # requested by cancel(), taken by run()
        self._cancelling: set[int] = set()  # resident slots whose budget was zeroed
        self.tiles_dev = None
        self.n_tiles = 0
        self._tiles_dirty = True
        # where the wall time of run() goes (seconds) and how full the steps were
        self.stats = {"steps": 0, "t_admit": 0.0, "t_upload": 0.0, "t_init": 0.0, "t_step": 0.0,
                      "t_wait": 0.0, "t_retire": 0.0, "t_idle": 0.0, "active_sum": 0,
                      "tiles_sum": 0}

    # ------------------------------------------------------------------ slots
    def _set_dummy(self, s: int) -> None:
        off = self.dummy_base + s * 3 * DUMMY_L ** 3
        self.table[s] = (off, off, 1, 1, DUMMY_L, 1, 0, 0, 0, 0)

    @staticmethod
    def _stage(ring: PinnedRing, arr: np.ndarray) -> tuple[torch.Tensor, int]:
        """arr copied into the ring's next pinned buffer: (host tensor view, buffer)."""
        a = np.ascontiguousarray(arr)
        buf, k = ring.take()
        view = buf[:a.nbytes]
        view.numpy()[:] = a.reshape(-1).view(np.uint8)
        return view.view(torch.from_numpy(a[:0]).dtype).reshape(a.shape), k

    def _to_dev(self, arr: np.ndarray, ring: PinnedRing | None = None) -> torch.Tensor:
        """Host array -> new device tensor through pinned memory, without waiting for the
        stream."""
        ring = ring or self._h2d
        host, k = self._stage(ring, arr)
        out = torch.empty(host.shape, dtype=host.dtype, device=self.device)
        out.copy_(host, non_blocking=True)
        ring.guard(k)
        return out

    def _upload_table(self) -> None:
        check(lib().hsg_batch_check(self.table.ctypes.data_as(ctypes.c_void_p), self.n_slots,
                                    self.spins.numel(), self.J.numel()))
        host, k = self._stage(self._h2d, self.table.view(np.uint8))
        self.chains.copy_(host, non_blocking=True)
        self._h2d.guard(k)

    @property
    def capacity_elements(self) -> int:
        """Elements of the spin arena (the coupling arena is as large)."""
        return self.arena_s.size

    def cancel(self, rid: int) -> None:
        """Cancel request rid (thread-safe; takes effect at the next scheduling step).
        A request not yet admitted returns at once with status "cancelled" and NaN
        results; a resident one stops sweeping and returns its energy and magnetisation
        after the sweeps done so far; one already finished is not affected."""
        with self._cancel_lock:
            self._cancel_ids.add(int(rid))

    def _take_cancels(self, pending: deque, queue: deque, t: float) -> list[Result]:
        with self._cancel_lock:
            ids, self._cancel_ids = self._cancel_ids, set()
        if not ids:
            return []
        out = []
        for dq in (pending, queue):
            keep = [r for r in dq if r.rid not in ids]
            for r in dq:
                if r.rid in ids:
                    out.append(Result(r.rid, math.nan, np.full(3, math.nan), r.arrival, t, t,
                                      status="cancelled"))
            dq.clear()
            dq.extend(keep)
        slots = [sl for sl, v in self.active.items()
                 if v[0].rid in ids and sl not in self._cancelling]
        if slots:
            idx = self._to_dev(np.asarray(slots, dtype=np.int64))
            self.remaining.index_fill_(0, idx, 0)  # the next step sweeps them no more
            self._cancelling.update(slots)
        return out

    def footprint(self, req: Request) -> int:
        return 2 * 3 * req.spins * self.es

    def try_admit(self, req: Request, now: float) -> bool:
        if not self.free_slots:
            return False
        if not (2 <= req.L <= BATCH_L_MAX and req.L % 2 == 0):
            raise ValueError(f"request {req.rid}: L={req.L} not servable")
        n = 3 * req.spins
        s_off = self.arena_s.alloc(n)
        if s_off is None:
            return False
        j_off = self.arena_j.alloc(n)
        if j_off is None:
            self.arena_s.release(s_off, n)
            return False
        slot = self.free_slots.pop()
        self.table[slot] = (s_off, j_off, req.seed, req.seed, req.L, req.k, 0, 0, HSG_CHAIN_INIT_J,
                            0)
        self.active[slot] = (req, s_off, j_off, now, self._it)
        return True

    def _init_new(self, slots: list[int]) -> None:
        """Philox initial state (spins and couplings from the request seed) of newly
        admitted lattices, through a small batch that views the same buffers."""
        if not slots:
            return
        sub = self.table[slots].copy()
        n = len(slots)
        dev = self.device
        chains = self._to_dev(sub.view(np.uint8))
        E = torch.zeros(n, dtype=torch.float64, device=dev)
        zeros = torch.zeros(n, dtype=torch.int32, device=dev)
        order = torch.arange(n, dtype=torch.int32, device=dev)
        beta = torch.zeros(n, dtype=torch.float64, device=dev)
        d = _Batch(n, _dtype_code(self.dtype), chains.data_ptr(), self.spins.data_ptr(),
                   self.J.data_ptr(), beta.data_ptr(), E.data_ptr(), zeros.data_ptr(), None,
                   order.data_ptr(), 256, 0)
        check(lib().hsg_batch_init(ctypes.byref(d), _stream(None)))
        idx = self._to_dev(np.asarray(slots, dtype=np.int64))
        self.E[idx] = E
        self.sweep_ctr.index_fill_(0, idx, 0)  # (a scalar assignment would wait for the stream)
        reqs = [self.active[s][0] for s in slots]
        self.remaining[idx] = self._to_dev(np.asarray([r.sweeps for r in reqs], dtype=np.int32))
        self.beta[idx] = self._to_dev(np.asarray([0.0 if math.isinf(r.T) else 1.0 / r.T
                                                  for r in reqs], dtype=np.float64))
        del chains, E, zeros, order, beta  # stream-ordered frees

    def _build_tiles(self) -> None:
        act = np.array(sorted(self.active), dtype=np.int32)
        cap = int(sum(-(-(self.table[s]["L"] ** 3 // 2) // self.tile_sites) for s in act)) + 1
        tiles = np.zeros(2 * cap, dtype=np.int32)
        n = ctypes.c_int32()
        check(lib().hsg_batch_tiles(self.table.ctypes.data_as(ctypes.c_void_p), self.n_slots,
                                    act.ctypes.data_as(ctypes.c_void_p), act.size, self.tile_sites,
                                    tiles.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(n)))
        self.n_tiles = n.value
        # a new tensor: the previous table may still be read by a step in flight
        need = 8 * n.value
        if self._tile_ring is None or self._tile_ring.nbytes < need:
            self._tile_ring = PinnedRing(4, max(need * 2, 1 << 16))
        self.tiles_dev = self._to_dev(tiles[:2 * n.value], self._tile_ring)
        self._tiles_dirty = False

    def step(self) -> None:
        """Advance every resident lattice by up to step_sweeps sweeps."""
        if self._tiles_dirty:
            self._build_tiles()
        if self.n_tiles == 0:
            return
        check(lib().hsg_batch_pass_sweep(ctypes.byref(self._d), _ptr(self.tiles_dev),
                                         self.n_tiles, self.tile_sites, 0, 0, self.step_sweeps,
                                         _stream(None)))

    def _begin_retire(self, done: list[int]) -> tuple:
        """Enqueue the read-back of finished lattices (magnetisation, tracked energy)
        into pinned memory and free their slots and memory at once: work enqueued later
        on the stream -- a new lattice's initial state -- runs after the read-back."""
        n = len(done)
        pairs = self._to_dev(np.asarray([[s, s] for s in done], dtype=np.int32))
        m_dev = torch.empty((n, 15), dtype=torch.float64, device=self.device)
        check(lib().hsg_batch_overlap(ctypes.byref(self._d), _ptr(pairs), n, _ptr(m_dev),
                                      _stream(None)))
        idx = self._to_dev(np.asarray(done, dtype=np.int64))
        buf, k = self._d2h.take()
        # m (3), E and the sweeps made per lattice
        both = buf[:40 * n].view(torch.float64).reshape(n, 5)
        m_E = torch.cat([m_dev[:, 9:12], self.E[idx].unsqueeze(1),
                         self.sweep_ctr[idx].double().unsqueeze(1)], dim=1)
        both.copy_(m_E, non_blocking=True)
        self._d2h.guard(k)
        ev = self._d2h.events[k]
        m_pin, E_pin = both[:, :3], both[:, 3:]
        info = []
        for s in done:
            req, s_off, j_off, t_adm, it_adm = self.active.pop(s)
            status = "cancelled" if s in self._cancelling else "ok"
            self._cancelling.discard(s)
            info.append((req, t_adm, it_adm, self._it, status))
            self.arena_s.release(s_off, 3 * req.spins)
            self.arena_j.release(j_off, 3 * req.spins)
            self._set_dummy(s)
            self.free_slots.append(s)
        self._tiles_dirty = True
        self._table_dirty = True
        return ev, info, m_pin, E_pin

    @staticmethod
    def _finish_retire(rec: tuple, t_done: float) -> list[Result]:
        ev, info, m_pin, E_pin = rec
        ev.synchronize()
        m, E = m_pin.numpy().copy(), E_pin.numpy().copy()
        return [Result(req.rid, float(E[i, 0]), m[i].copy(), req.arrival, t_adm, t_done, it_adm,
                       it_fin, status, int(E[i, 1]))
                for i, (req, t_adm, it_adm, it_fin, status) in enumerate(info)]

    # -------------------------------------------------------------------- loop
    def run(self, trace: list[Request], realtime: bool = True,
            on_iteration=None) -> list[Result]:
        """Serve a trace.  realtime=True releases each request at its arrival time
        (wall clock from the start of the run); False releases all at once.  A request
        that cannot be served (request_problem) returns at its arrival with status
        "rejected: ..." and does not affect the others; cancel() may be called from
        another thread, or from on_iteration(iteration, server), called after every
        scheduling step.

        Each iteration: admit what fits, enqueue one step for the resident lattices and
        a non-blocking copy of their remaining budgets, then wait for the PREVIOUS
        step's copy and retire the lattices it shows finished (their read-back is
        collected one iteration later)."""
        pending = deque(sorted(trace, key=lambda r: r.arrival))
        queue: deque[Request] = deque()
        results: list[Result] = []
        t0 = time.perf_counter()
        now = (lambda: time.perf_counter() - t0) if realtime else (lambda: 0.0)
        st = self.stats
        clock = time.perf_counter
        if not hasattr(self, "_rem_pin"):
            self._rem_pin = [torch.empty(self.n_slots, dtype=torch.int32).pin_memory()
                             for _ in range(2)]
        rem_pin = self._rem_pin
        prev = None       # (buffer, event, {slot: request id}) of the step in flight
        retiring = []     # (record, detection time) of read-backs in flight
        it = 0
        self._it = 0
        self._table_dirty = False
        while pending or queue or self.active or prev is not None or retiring:
            c0 = clock()
            t = now()
            results.extend(self._take_cancels(pending, queue, t))
            while pending and (not realtime or pending[0].arrival <= t):
                req = pending.popleft()
                why = request_problem(req, self.capacity_elements)
                if why is None:
                    queue.append(req)
                else:
                    results.append(Result(req.rid, math.nan, np.full(3, math.nan), req.arrival,
                                          t, t, status=f"rejected: {why}"))
            admitted = []
            while queue and self.try_admit(queue[0], now()):
                admitted.append(self._slot_of(queue.popleft()))
            ca = clock()
            if admitted or self._table_dirty:
                self._upload_table()
                self._table_dirty = False
            cb = clock()
            if admitted:
                self._init_new(admitted)
                self._tiles_dirty = True
            c1 = clock()
            st["t_admit"] += ca - c0
            st["t_upload"] += cb - ca
            st["t_init"] += c1 - cb
            cur = None
            if self.active:
                self.step()
                b = it & 1
                rem_pin[b].copy_(self.remaining, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record()
                cur = (b, ev, {s: v[0].rid for s, v in self.active.items()})
                st["steps"] += 1
                st["active_sum"] += len(self.active)
                st["tiles_sum"] += self.n_tiles
            c2 = clock()
            st["t_step"] += c2 - c1
            # read-backs enqueued last iteration: their step has finished by now
            for rec, t_det in retiring:
                results.extend(self._finish_retire(rec, t_det))
            retiring = []
            if prev is not None:
                b, ev, act = prev
                ev.synchronize()
                c3 = clock()
                st["t_wait"] += c3 - c2
                t_det = now()
                rem = rem_pin[b].numpy()
                done = [s for s, rid in act.items()
                        if rem[s] == 0 and s in self.active and self.active[s][0].rid == rid]
                if done:
                    retiring.append((self._begin_retire(done), t_det))
                st["t_retire"] += clock() - c3
            prev = cur
            it += 1
            self._it = it
            if on_iteration is not None:
                on_iteration(it, self)
            if prev is None and not retiring and not self.active:
                if queue:
                    raise RuntimeError(f"request {queue[0].rid} does not fit the HBM budget")
                c4 = clock()
                if pending and realtime:
                    time.sleep(max(0.0, pending[0].arrival - now()))
                st["t_idle"] += clock() - c4
        return results

    def _slot_of(self, req: Request) -> int:
        for s, (r, *_rest) in self.active.items():
            if r is req:
                return s
        raise KeyError(req.rid)


def latency_stats(results: list[Result]) -> dict:
    """Latency percentiles of the completed requests (status "ok"); cancelled and
    rejected ones are counted apart."""
    lat = np.array([r.latency for r in results if r.status == "ok"])
    out = {"n": int(lat.size), "cancelled": sum(r.status == "cancelled" for r in results),
           "rejected": sum(r.status.startswith("rejected") for r in results)}
    if lat.size:
        out.update({"p50_s": float(np.percentile(lat, 50)),
                    "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean()),
                    "max_s": float(lat.max())})
    return out
