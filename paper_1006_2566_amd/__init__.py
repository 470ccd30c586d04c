"""Heisenberg spin-glass Monte Carlo on AMD MI355X (gfx950).

Python binding of ``libhsg.so`` (C interface in ``include/hsg.h``).  This module
only marshals arguments: every step of a sweep runs in the HIP kernels of the
library.  PyTorch provides device memory and the current HIP stream.

The model and dynamics are those of Bernaschi, Parisi & Parisi, "The Heisenberg spin
glass model on GPU: myths and actual facts" (arXiv:1006.2566): 3-component unit spins
on an L^3 periodic lattice with Gaussian couplings (§2, eqs. 1-2), checkerboard
updates with over-relaxation (§4), plus the Metropolis / heat-bath moves the paper
names, driven by a Philox counter-based generator.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

__all__ = ["Lattice", "HsgError", "lib", "lattice_bytes", "LIB_PATH"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhsg.so")

HSG_F32, HSG_F64 = 0, 1
HSG_HEAT_BATH = 1
HSG_SNAKE = 2
HSG_FUSED = 4
HSG_MARCH_PHASE = 16
HSG_PLANE_LAUNCH = 32
HSG_STREAM_LOADS = 64
HSG_PHASE_LAUNCH = 128
HSG_PHASE_MC = 256
# launch kinds reported by hsg_sweep_timed
LAUNCH_OTHER, LAUNCH_MC_PASS, LAUNCH_OR_PASS, LAUNCH_OR_PHASE, LAUNCH_OR_PHASE_MC, \
    LAUNCH_MARCH = range(6)
LAUNCH_NAMES = ("other", "mc_pass", "or_pass", "or_phase", "or_phase_mc", "march")
FUSED_MIN_L, FUSED_MAX_L = 256, 1024
PHASE_MIN_L, PHASE_MAX_L = 64, 1024
FOURIER_VALUES = 65
L_MAX = 1290


def fused_supported(L: int) -> bool:
    """Whether HSG_FUSED takes effect for an L^3 lattice."""
    return FUSED_MIN_L <= L <= FUSED_MAX_L and L % 64 == 0


def phase_supported(L: int) -> bool:
    """Whether HSG_PHASE_LAUNCH takes effect for an L^3 lattice (L a multiple of 64 with
    64 <= L <= 1024: the launch's 32-bit element offsets reach 3 L^3)."""
    return PHASE_MIN_L <= L <= PHASE_MAX_L and L % 64 == 0


def default_flags(L: int, dtype=None) -> int:
    """Traversal flags of a sweep that names none: Monte Carlo passes one launch each in
    alternating z order, over-relaxation phases as one launch each where the lattice
    gives that launch enough workgroups (L >= 256) -- in binary32 with the next sweep's
    colour-0 Monte Carlo pass in the same launch -- which measures fastest on MI355X
    (HSG_FUSED is opt-in).  Spins are the same either way."""
    if not (L >= 256 and phase_supported(L)):
        return HSG_SNAKE
    f64 = dtype is not None and str(dtype) in ("torch.float64", "float64")
    return HSG_SNAKE | (HSG_PHASE_LAUNCH if f64 else HSG_PHASE_MC)


class HsgError(RuntimeError):
    """A libhsg call returned an error status."""

    def __init__(self, code: int, message: str):
        super().__init__(f"libhsg error {code}: {message}")
        self.code = code


class _Lattice(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("dtype", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("sweep", ctypes.c_uint64), ("spins", ctypes.c_void_p), ("J", ctypes.c_void_p),
                ("E", ctypes.c_void_p), ("work", ctypes.c_void_p), ("work_bytes", ctypes.c_size_t)]


class _SweepParams(ctypes.Structure):
    _fields_ = [("T", ctypes.c_double), ("k_hits", ctypes.c_int32), ("n_or", ctypes.c_int32),
                ("renorm_every", ctypes.c_int32), ("flags", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded HIP library.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing; build it with "
                              "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)
        LP = ctypes.POINTER(_Lattice)
        L.hsg_lattice_bytes.argtypes = [I32, I32, SZ, SZ, SZ]
        L.hsg_init_lattice.argtypes = [LP, P]
        L.hsg_import.argtypes = [LP, P, P, P]
        L.hsg_export.argtypes = [LP, P, P, P]
        L.hsg_sweep.argtypes = [LP, ctypes.POINTER(_SweepParams), I32, P]
        L.hsg_sweep_timed.argtypes = [LP, ctypes.POINTER(_SweepParams), I32, P, I32, P, P,
                                      ctypes.POINTER(I32)]
        L.hsg_sweep_noalloc.argtypes = [LP, ctypes.POINTER(_SweepParams), I32, P]
        L.hsg_energy.argtypes = [LP, I32, P, P]
        L.hsg_overlap.argtypes = [LP, LP, P, P]
        L.hsg_overlap_fourier.argtypes = [LP, LP, P, P]
        L.hsg_last_error.restype = ctypes.c_char_p
        for name in ("hsg_lattice_bytes", "hsg_init_lattice", "hsg_import", "hsg_export",
                     "hsg_sweep", "hsg_sweep_timed", "hsg_sweep_noalloc", "hsg_energy",
                     "hsg_overlap",
                     "hsg_overlap_fourier"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != 0:
        raise HsgError(rc, lib().hsg_last_error().decode())


def _dtype_code(dtype: torch.dtype) -> int:
    if dtype == torch.float32:
        return HSG_F32
    if dtype == torch.float64:
        return HSG_F64
    raise TypeError(f"spins are float32 or float64, not {dtype}")


def lattice_bytes(L: int, dtype: torch.dtype = torch.float32) -> tuple[int, int, int]:
    """(spin_bytes, J_bytes, work_bytes) of an L^3 lattice."""
    s, j, w = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    check(lib().hsg_lattice_bytes(L, _dtype_code(dtype), ctypes.byref(s), ctypes.byref(j),
                                  ctypes.byref(w)))
    return s.value, j.value, w.value


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class Lattice:
    """One L^3 lattice resident on the GPU (colour-split layout, see include/hsg.h).

    ``init="random"`` draws the Philox initial state from ``seed``; ``init=None``
    leaves the buffers for :meth:`load`.
    """

    def __init__(self, L: int, dtype: torch.dtype = torch.float32, seed: int = 1,
                 device: str | torch.device = "cuda", init: str | None = "random",
                 stream=None):
        spin_b, j_b, work_b = lattice_bytes(L, dtype)
        self.L, self.dtype, self.device = L, dtype, torch.device(device)
        n = 3 * L ** 3
        self.spins = torch.empty(n, dtype=dtype, device=self.device)
        self.J = torch.empty(n, dtype=dtype, device=self.device)
        self.E = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.work = torch.zeros(work_b, dtype=torch.uint8, device=self.device)
        self._d = _Lattice(L, _dtype_code(dtype), seed & (2 ** 64 - 1), 0, self.spins.data_ptr(),
                           self.J.data_ptr(), self.E.data_ptr(), self.work.data_ptr(), work_b)
        if init == "random":
            self.init_random(stream)

    # ------------------------------------------------------------------ state
    @property
    def N(self) -> int:
        return self.L ** 3

    @property
    def seed(self) -> int:
        return self._d.seed

    @property
    def sweep_index(self) -> int:
        return self._d.sweep

    @sweep_index.setter
    def sweep_index(self, value: int) -> None:
        self._d.sweep = int(value)

    def init_random(self, stream=None) -> None:
        check(lib().hsg_init_lattice(ctypes.byref(self._d), _stream(stream)))

    def load(self, spins, J=None, stream=None) -> None:
        """Load canonical-layout spins (and couplings), shape (3, N), any device."""
        s = torch.as_tensor(spins).to(device=self.device, dtype=self.dtype).contiguous()
        assert s.numel() == 3 * self.N
        j = None
        if J is not None:
            j = torch.as_tensor(J).to(device=self.device, dtype=self.dtype).contiguous()
            assert j.numel() == 3 * self.N
        check(lib().hsg_import(ctypes.byref(self._d), _ptr(s), _ptr(j) if j is not None else None,
                               _stream(stream)))
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()

    def export(self, stream=None) -> tuple[torch.Tensor, torch.Tensor]:
        """Canonical-layout (spins, J), each of shape (3, N), on the device."""
        s = torch.empty((3, self.N), dtype=self.dtype, device=self.device)
        j = torch.empty((3, self.N), dtype=self.dtype, device=self.device)
        check(lib().hsg_export(ctypes.byref(self._d), _ptr(s), _ptr(j), _stream(stream)))
        return s, j

    # --------------------------------------------------------------- dynamics
    def sweep(self, T: float, k: int = 1, n_or: int = 0, renorm_every: int = 0,
              n_sweeps: int = 1, heat_bath: bool = False, flags: int | None = None,
              stream=None) -> None:
        """n_sweeps sweeps; flags None = default_flags(L, dtype)."""
        f = default_flags(self.L, self.dtype) if flags is None else int(flags)
        p = _SweepParams(float(T), int(k), int(n_or), int(renorm_every),
                         (HSG_HEAT_BATH if heat_bath else 0) | f)
        check(lib().hsg_sweep(ctypes.byref(self._d), ctypes.byref(p), int(n_sweeps),
                              _stream(stream)))

    def sweep_timed(self, T: float, k: int = 1, n_or: int = 0, renorm_every: int = 0,
                    n_sweeps: int = 1, heat_bath: bool = False, flags: int | None = None,
                    capacity: int = 4096, stream=None) -> list[tuple[int, float]]:
        """As sweep(), with every launch timed by HIP events on the launch stream:
        [(launch kind, ms)] in launch order (hsg_sweep_timed; waits for the stream)."""
        import numpy as np
        f = default_flags(self.L, self.dtype) if flags is None else int(flags)
        p = _SweepParams(float(T), int(k), int(n_or), int(renorm_every),
                         (HSG_HEAT_BATH if heat_bath else 0) | f)
        kinds = np.zeros(capacity, dtype=np.int32)
        ms = np.zeros(capacity, dtype=np.float32)
        n = ctypes.c_int32()
        check(lib().hsg_sweep_timed(ctypes.byref(self._d), ctypes.byref(p), int(n_sweeps),
                                    _stream(stream), capacity, kinds.ctypes.data_as(ctypes.c_void_p),
                                    ms.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
        return [(int(kinds[i]), float(ms[i])) for i in range(n.value)]

    # ---------------------------------------------------------- observables
    def energy(self, recompute: bool = False, stream=None) -> torch.Tensor:
        """Energy H as a 1-element float64 device tensor (tracked or recomputed)."""
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        check(lib().hsg_energy(ctypes.byref(self._d), int(bool(recompute)), _ptr(out),
                               _stream(stream)))
        return out

    def overlap(self, other: "Lattice", stream=None) -> torch.Tensor:
        """15 float64 values: Q[3x3] row-major, then m_self[3], m_other[3]."""
        out = torch.empty(15, dtype=torch.float64, device=self.device)
        check(lib().hsg_overlap(ctypes.byref(self._d), ctypes.byref(other._d), _ptr(out),
                                _stream(stream)))
        return out

    def overlap_fourier(self, other: "Lattice", out: torch.Tensor | None = None,
                        stream=None) -> torch.Tensor:
        """The 65-value record of hsg_overlap_fourier: Q(0) (9), Re/Im Q(k_d) for
        d = x, y, z (18 each), q2(0), q2(k_min)."""
        if out is None:
            out = torch.empty(FOURIER_VALUES, dtype=torch.float64, device=self.device)
        check(lib().hsg_overlap_fourier(ctypes.byref(self._d), ctypes.byref(other._d),
                                        _ptr(out), _stream(stream)))
        return out


def beta(T: float) -> float:
    return 0.0 if math.isinf(T) else 1.0 / T
