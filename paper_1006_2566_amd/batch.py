"""Batched form: many lattices ("chains") of mixed size, replicas and parallel-tempering
ladders advanced by one persistent launch of ``hsg_batch_sweep``.

Only argument marshalling lives here: the chain table, ladders and work order are
built on the host, every sweep, exchange and overlap runs in libhsg's kernels.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math

import numpy as np
import torch

from . import (FOURIER_VALUES, HSG_F32, HSG_F64, HSG_HEAT_BATH, _dtype_code, _Lattice, _ptr,
               _stream, check, lib)

HSG_CHAIN_INIT_J = 8
BATCH_L_MAX = 256

CHAIN_DTYPE = np.dtype([("spin_offset", "<i8"), ("J_offset", "<i8"), ("seed", "<u8"),
                        ("J_seed", "<u8"), ("L", "<i4"), ("k_hits", "<i4"), ("n_or", "<i4"),
                        ("renorm_every", "<i4"), ("flags", "<i4"), ("reserved", "<i4")])
assert CHAIN_DTYPE.itemsize == 56


class _Batch(ctypes.Structure):
    _fields_ = [("n_chains", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("chains", ctypes.c_void_p), ("spins", ctypes.c_void_p), ("J", ctypes.c_void_p),
                ("beta", ctypes.c_void_p), ("E", ctypes.c_void_p), ("sweep", ctypes.c_void_p),
                ("remaining", ctypes.c_void_p), ("order", ctypes.c_void_p),
                ("threads", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _PT(ctypes.Structure):
    _fields_ = [("n_ladders", ctypes.c_int32), ("n_temps", ctypes.c_int32),
                ("chain_at_slot", ctypes.c_void_p), ("beta_of_slot", ctypes.c_void_p),
                ("accepted", ctypes.c_void_p), ("round", ctypes.c_void_p),
                ("seed", ctypes.c_uint64)]


_bound = False


def _bind():
    global _bound
    if _bound:
        return
    L = lib()
    P, I32 = ctypes.c_void_p, ctypes.c_int32
    BP, PP = ctypes.POINTER(_Batch), ctypes.POINTER(_PT)
    L.hsg_batch_check.argtypes = [P, I32, ctypes.c_int64, ctypes.c_int64]
    L.hsg_batch_init.argtypes = [BP, P]
    L.hsg_batch_sweep.argtypes = [BP, I32, P]
    L.hsg_batch_energy.argtypes = [BP, P, P]
    L.hsg_batch_overlap.argtypes = [BP, P, I32, P, P]
    L.hsg_pt_exchange.argtypes = [PP, BP, P]
    L.hsg_pt_overlap.argtypes = [PP, BP, P, I32, P, P]
    L.hsg_batch_overlap_fourier.argtypes = [BP, P, I32, P, P]
    L.hsg_pt_overlap_fourier.argtypes = [PP, BP, P, I32, P, P]
    for name in ("hsg_batch_check", "hsg_batch_init", "hsg_batch_sweep",
                 "hsg_batch_energy", "hsg_batch_overlap", "hsg_pt_exchange", "hsg_pt_overlap",
                 "hsg_batch_overlap_fourier", "hsg_pt_overlap_fourier"):
        getattr(L, name).restype = ctypes.c_int
    _bound = True


@dataclasses.dataclass
class ChainSpec:
    """One chain: lattice size, seeds, dynamics and temperature.  Chains with the same
    ``J_group`` share one block of couplings (one disorder sample)."""
    L: int
    seed: int
    J_group: int
    J_seed: int
    T: float = 1.0
    k: int = 1
    n_or: int = 0
    renorm_every: int = 0
    heat_bath: bool = False


def lpt_order(Ls, groups) -> np.ndarray:
    """Work order: largest lattices first (longest-processing-time rule), chains of
    one coupling group next to each other."""
    Ls = np.asarray(Ls)
    groups = np.asarray(groups)
    return np.lexsort((np.arange(Ls.size), groups, -Ls.astype(np.int64) ** 3)).astype(np.int32)


class Batch:
    """Chains resident on the GPU, advanced together by ``sweep``."""

    def __init__(self, specs: list[ChainSpec], dtype: torch.dtype = torch.float32,
                 device: str | torch.device = "cuda", threads: int = 256,
                 order: np.ndarray | None = None, init: bool = True, track_remaining=False,
                 stream=None):
        _bind()
        self.specs = list(specs)
        self.n = len(self.specs)
        self.dtype, self.device = dtype, torch.device(device)
        table = np.zeros(self.n, dtype=CHAIN_DTYPE)
        spin_off = 0
        group_off: dict[int, tuple[int, int]] = {}
        J_off = 0
        for i, c in enumerate(self.specs):
            if c.L % 2 or not 2 <= c.L <= BATCH_L_MAX:
                raise ValueError(f"chain {i}: L={c.L} must be even and <= {BATCH_L_MAX}")
            n_el = 3 * c.L ** 3
            flags = HSG_HEAT_BATH if c.heat_bath else 0
            if c.J_group not in group_off:
                group_off[c.J_group] = (J_off, c.L)
                J_off += n_el
                flags |= HSG_CHAIN_INIT_J
            off, gL = group_off[c.J_group]
            if gL != c.L:
                raise ValueError(f"chain {i}: coupling group {c.J_group} has L={gL}, not {c.L}")
            table[i] = (spin_off, off, c.seed & (2 ** 64 - 1), c.J_seed & (2 ** 64 - 1), c.L, c.k,
                        c.n_or, c.renorm_every, flags, 0)
            spin_off += n_el
        self.spin_elems, self.J_elems = spin_off, J_off
        self.table = table
        check(lib().hsg_batch_check(table.ctypes.data_as(ctypes.c_void_p), self.n, spin_off, J_off))
        dev = self.device
        self.chains = torch.from_numpy(table.view(np.uint8).copy()).to(dev)
        self.spins = torch.empty(spin_off, dtype=dtype, device=dev)
        self.J = torch.empty(J_off, dtype=dtype, device=dev)
        betas = [0.0 if math.isinf(c.T) else 1.0 / c.T for c in self.specs]
        self.beta = torch.tensor(betas, dtype=torch.float64, device=dev)
        self.E = torch.zeros(self.n, dtype=torch.float64, device=dev)
        self.sweep_ctr = torch.zeros(self.n, dtype=torch.int32, device=dev)
        self.remaining = (torch.zeros(self.n, dtype=torch.int32, device=dev)
                          if track_remaining else None)
        if order is None:
            order = lpt_order([c.L for c in self.specs], [c.J_group for c in self.specs])
        if not np.array_equal(np.sort(np.asarray(order)), np.arange(self.n)):
            raise ValueError("order must be a permutation of the chain indices")
        self.order = torch.from_numpy(np.ascontiguousarray(order, dtype=np.int32)).to(dev)
        self._d = _Batch(self.n, _dtype_code(dtype), self.chains.data_ptr(), self.spins.data_ptr(),
                         self.J.data_ptr(), self.beta.data_ptr(), self.E.data_ptr(),
                         self.sweep_ctr.data_ptr(),
                         self.remaining.data_ptr() if self.remaining is not None else None,
                         self.order.data_ptr(), threads, 0)
        self._export_work: dict[int, torch.Tensor] = {}
        if init:
            self.init(stream)

    @property
    def threads(self) -> int:
        return self._d.threads

    @threads.setter
    def threads(self, v: int) -> None:
        self._d.threads = int(v)

    def init(self, stream=None) -> None:
        check(lib().hsg_batch_init(ctypes.byref(self._d), _stream(stream)))

    def sweep(self, n_sweeps: int, stream=None) -> None:
        check(lib().hsg_batch_sweep(ctypes.byref(self._d), int(n_sweeps), _stream(stream)))

    def energies(self, recompute: bool = False, stream=None) -> torch.Tensor:
        if not recompute:
            return self.E.clone()
        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        check(lib().hsg_batch_energy(ctypes.byref(self._d), _ptr(out), _stream(stream)))
        return out

    def overlap(self, pairs, stream=None) -> torch.Tensor:
        p = torch.as_tensor(np.asarray(pairs, dtype=np.int32).reshape(-1, 2)).to(self.device)
        out = torch.empty((p.shape[0], 15), dtype=torch.float64, device=self.device)
        check(lib().hsg_batch_overlap(ctypes.byref(self._d), _ptr(p), p.shape[0], _ptr(out),
                                      _stream(stream)))
        return out

    def overlap_fourier(self, pairs, stream=None) -> torch.Tensor:
        """Records of hsg_batch_overlap_fourier, shape (n_pairs, 65)."""
        p = torch.as_tensor(np.asarray(pairs, dtype=np.int32).reshape(-1, 2)).to(self.device)
        out = torch.empty((p.shape[0], FOURIER_VALUES), dtype=torch.float64, device=self.device)
        check(lib().hsg_batch_overlap_fourier(ctypes.byref(self._d), _ptr(p), p.shape[0],
                                              _ptr(out), _stream(stream)))
        return out

    def chain_offsets(self, c: int) -> tuple[int, int]:
        return int(self.table[c]["spin_offset"]), int(self.table[c]["J_offset"])

    def _chain_lattice(self, c: int) -> _Lattice:
        """A single-lattice descriptor viewing chain c's buffers (and its energy slot)."""
        from . import lattice_bytes
        c = int(c)
        L = int(self.table[c]["L"])
        so, jo = self.chain_offsets(c)
        if L not in self._export_work:
            self._export_work[L] = torch.zeros(lattice_bytes(L, self.dtype)[2], dtype=torch.uint8,
                                               device=self.device)
        w = self._export_work[L]
        es = self.spins.element_size()
        return _Lattice(L, _dtype_code(self.dtype), int(self.table[c]["seed"]), 0,
                        self.spins.data_ptr() + so * es, self.J.data_ptr() + jo * es,
                        self.E.data_ptr() + 8 * c, w.data_ptr(), w.numel())

    def export_chain(self, c: int, stream=None) -> tuple[torch.Tensor, torch.Tensor]:
        """Canonical (spins, J) of chain c, via hsg_export on a view of its buffers."""
        d = self._chain_lattice(c)
        L = d.L
        s = torch.empty((3, L ** 3), dtype=self.dtype, device=self.device)
        j = torch.empty((3, L ** 3), dtype=self.dtype, device=self.device)
        check(lib().hsg_export(ctypes.byref(d), _ptr(s), _ptr(j), _stream(stream)))
        return s, j

    def load_chain(self, c: int, spins, J=None, stream=None) -> None:
        """Load canonical-layout spins (and couplings, which chains of one group share)
        into chain c via hsg_import; its tracked energy becomes H."""
        d = self._chain_lattice(c)
        n = 3 * d.L ** 3
        s = torch.as_tensor(spins).to(device=self.device, dtype=self.dtype).contiguous()
        assert s.numel() == n
        j = None
        if J is not None:
            j = torch.as_tensor(J).to(device=self.device, dtype=self.dtype).contiguous()
            assert j.numel() == n
        check(lib().hsg_import(ctypes.byref(d), _ptr(s), _ptr(j) if j is not None else None,
                               _stream(stream)))
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()


class Tempering:
    """Parallel-tempering ladders over chains of a batch: ``ladders[l, t]`` is the chain
    first placed in slot t (inverse temperature ``betas[t]``) of ladder l."""

    def __init__(self, batch: Batch, ladders, betas, seed: int, stream=None):
        _bind()
        self.batch = batch
        lad = np.ascontiguousarray(ladders, dtype=np.int32)
        self.n_ladders, self.n_temps = lad.shape
        dev = batch.device
        self.chain_at_slot = torch.from_numpy(lad.copy()).to(dev)
        self.beta_of_slot = torch.tensor(np.asarray(betas, dtype=np.float64), device=dev)
        self.accepted = torch.zeros(lad.shape, dtype=torch.int32, device=dev)
        self.round = torch.zeros(1, dtype=torch.int32, device=dev)
        self._d = _PT(self.n_ladders, self.n_temps, self.chain_at_slot.data_ptr(),
                      self.beta_of_slot.data_ptr(), self.accepted.data_ptr(),
                      self.round.data_ptr(), seed & (2 ** 64 - 1))
        # every chain of a ladder starts at its slot's temperature
        flat = self.chain_at_slot.reshape(-1).long()
        batch.beta[flat] = self.beta_of_slot.repeat(self.n_ladders)

    def exchange(self, stream=None) -> None:
        check(lib().hsg_pt_exchange(ctypes.byref(self._d), ctypes.byref(self.batch._d),
                                    _stream(stream)))

    def _pairs(self, ladder_pairs) -> torch.Tensor:
        if isinstance(ladder_pairs, torch.Tensor):
            return ladder_pairs.to(device=self.batch.device, dtype=torch.int32).reshape(-1, 2)
        return torch.as_tensor(np.asarray(ladder_pairs, dtype=np.int32).reshape(-1, 2)).to(
            self.batch.device)

    def overlap(self, ladder_pairs, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        p = self._pairs(ladder_pairs)
        if out is None:
            out = torch.empty((p.shape[0], self.n_temps, 15), dtype=torch.float64,
                              device=self.batch.device)
        check(lib().hsg_pt_overlap(ctypes.byref(self._d), ctypes.byref(self.batch._d), _ptr(p),
                                   p.shape[0], _ptr(out), _stream(stream)))
        return out

    def overlap_fourier(self, ladder_pairs, out: torch.Tensor | None = None,
                        stream=None) -> torch.Tensor:
        """Records of hsg_pt_overlap_fourier, shape (n_pairs, n_temps, 65)."""
        p = self._pairs(ladder_pairs)
        if out is None:
            out = torch.empty((p.shape[0], self.n_temps, FOURIER_VALUES), dtype=torch.float64,
                              device=self.batch.device)
        check(lib().hsg_pt_overlap_fourier(ctypes.byref(self._d), ctypes.byref(self.batch._d),
                                           _ptr(p), p.shape[0], _ptr(out), _stream(stream)))
        return out


def geometric_ladder(T_min: float, T_max: float, n: int) -> np.ndarray:
    """T_t = T_min (T_max / T_min)^(t / (n-1)), t = 0..n-1 (returned as inverse temperatures)."""
    t = np.arange(n, dtype=np.float64)
    T = T_min * (T_max / T_min) ** (t / max(n - 1, 1))
    return 1.0 / T


def pt_workload(n_samples: int = 256, Ls=(16, 24, 32, 48), replicas: int = 2, n_temps: int = 24,
                T_min: float = 0.12, T_max: float = 0.5, k: int = 4, base_seed: int = 1):
    """The batched workload: n_samples disorder samples with L drawn uniformly from Ls,
    `replicas` replicas each with an n_temps geometric temperature ladder; binary32,
    Metropolis with k hits, no over-relaxation.  Seeds from numpy's PCG64 on base_seed.

    Returns (specs, ladders [samples*replicas, n_temps], betas, pairs of ladders)."""
    rng = np.random.default_rng(base_seed)
    sample_L = rng.choice(np.asarray(Ls), size=n_samples)
    J_seeds = rng.integers(1, 2 ** 63, size=n_samples, dtype=np.int64)
    chain_seeds = rng.integers(1, 2 ** 63, size=(n_samples, replicas, n_temps), dtype=np.int64)
    betas = geometric_ladder(T_min, T_max, n_temps)
    specs, ladders, pairs = [], [], []
    for s in range(n_samples):
        first_ladder = len(ladders)
        for r in range(replicas):
            lad = []
            for t in range(n_temps):
                lad.append(len(specs))
                specs.append(ChainSpec(L=int(sample_L[s]), seed=int(chain_seeds[s, r, t]),
                                       J_group=s, J_seed=int(J_seeds[s]), T=1.0 / betas[t], k=k))
            ladders.append(lad)
        for r in range(1, replicas):
            pairs.append((first_ladder, first_ladder + r))
    return specs, np.asarray(ladders, dtype=np.int32), betas, np.asarray(pairs, dtype=np.int32)


class PTRunner:
    """Runs the tempering schedule: blocks of `sweeps_per_exchange` sweeps, each
    followed by one exchange round, and an overlap measurement every
    `exchanges_per_measure` rounds.  The measurement cycle is captured once in a HIP
    graph (torch.cuda.CUDAGraph) and replayed."""

    def __init__(self, batch: Batch, pt: Tempering, ladder_pairs, sweeps_per_exchange: int = 10,
                 exchanges_per_measure: int = 10, use_graph: bool = True, fourier: bool = False):
        self.batch, self.pt = batch, pt
        self.pairs = torch.as_tensor(np.asarray(ladder_pairs, dtype=np.int32).reshape(-1, 2)).to(
            batch.device)
        self.spe, self.epm = sweeps_per_exchange, exchanges_per_measure
        self.q = torch.zeros((self.pairs.shape[0], pt.n_temps, 15), dtype=torch.float64,
                             device=batch.device)
        # with fourier=True each cycle also writes the Fourier-overlap records, and
        # accumulate() adds them to the running moments of q2
        self.qk = None
        self.moments = None
        if fourier:
            from .observables import OverlapMoments
            self.qk = torch.zeros((self.pairs.shape[0], pt.n_temps, FOURIER_VALUES),
                                  dtype=torch.float64, device=batch.device)
            self.moments = OverlapMoments((self.pairs.shape[0], pt.n_temps))
        self.use_graph = use_graph
        self.graph = None

    def _cycle(self) -> None:
        for _ in range(self.epm):
            self.batch.sweep(self.spe)
            self.pt.exchange()
        self.pt.overlap(self.pairs, out=self.q)
        if self.qk is not None:
            self.pt.overlap_fourier(self.pairs, out=self.qk)

    def accumulate(self) -> None:
        """Adds the last cycle's Fourier records to the moments (copies them to the
        host, so the stream is synchronised)."""
        if self.moments is None:
            raise ValueError("PTRunner was built without fourier=True")
        self.moments.add(self.qk)

    def L_of_pair(self) -> np.ndarray:
        """Lattice size of each ladder pair (its first ladder's first chain)."""
        lad = self.pt.chain_at_slot.cpu().numpy()
        pairs = self.pairs.cpu().numpy()
        return np.array([self.batch.specs[int(lad[a, 0])].L for a, _ in pairs])

    def capture(self) -> None:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                self._cycle()
        torch.cuda.current_stream().wait_stream(s)
        self.graph = g

    @property
    def sweeps_per_cycle(self) -> int:
        return self.spe * self.epm

    def run_cycle(self) -> None:
        """One measurement cycle.  With graphs, the first cycle runs eagerly (it also
        loads every kernel) and is then captured; later cycles replay the graph."""
        if not self.use_graph:
            self._cycle()
        elif self.graph is None:
            self._cycle()
            self.capture()
        else:
            self.graph.replay()
