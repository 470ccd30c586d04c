"""Python shim over the plain CPU oracle (``oracle/libhsgo.so``).

TEST INFRASTRUCTURE ONLY.  This package defines what the GPU library must compute
for the checkerboard Monte Carlo sweep of the 3D Heisenberg spin glass
(Bernaschi, Parisi & Parisi, arXiv:1006.2566): the Hamiltonian of §2 eq. (1), the
local field of §2 eq. (2), over-relaxation and the checkerboard schedule of §4,
and the Metropolis / heat-bath / Philox / replica-exchange steps the paper names
but leaves to the reader.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it; the GPU library never does.

Arrays use the canonical layout: site ``i = x + L*y + L*L*z``; spins and couplings
are ``(3, N)`` arrays (component or bond direction first), ``J[d, i]`` being the
coupling on the bond ``(i, i + e_d)``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

TAG_MH, TAG_INIT_SPIN, TAG_INIT_J, TAG_PT, TAG_HB = 0, 1, 2, 3, 5

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_U32 = ctypes.c_uint32
_U64 = ctypes.c_uint64
_D = ctypes.c_double


def lib():
    """Load (building first if needed) the oracle library."""
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.hsgo_philox_many.argtypes = [_I64, _P, _P, _P]
        L.hsgo_u01_many.argtypes = [_I64, _P, _P]
        L.hsgo_poly_coefs_f64.argtypes = [_P]
        L.hsgo_poly_coefs_f32.argtypes = [_P]
        L.hsgo_pt_swap.argtypes = [_I32, _P, _P, _P, _U64, _U32, _U32, _P]
        L.hsgo_pt_swap.restype = ctypes.c_int
        L.hsgo_threads.restype = ctypes.c_int
        L.hsgo_set_threads.argtypes = [ctypes.c_int]
        for suf, real in (("f32", ctypes.c_float), ("f64", ctypes.c_double)):
            getattr(L, f"hsgo_sincos_2pi_{suf}").argtypes = [real, _P, _P]
            getattr(L, f"hsgo_trial_spin_{suf}").argtypes = [real, real, _P]
            getattr(L, f"hsgo_init_{suf}").argtypes = [_I32, _U64, _P, _P]
            getattr(L, f"hsgo_local_field_{suf}").argtypes = [_I32, _P, _P, _I32, _I32, _I32, _P]
            getattr(L, f"hsgo_overrelax_site_{suf}").argtypes = [_P, _P]
            getattr(L, f"hsgo_field_{suf}").argtypes = [_P, _P, _P]
            fn = getattr(L, f"hsgo_site_update_{suf}")
            fn.argtypes = [_I32, _P, _P, _U64, _U64, _U32, _U32, _I32, _D, _D, _P, _P]
            fn.restype = _I64
            getattr(L, f"hsgo_elem_many_{suf}").argtypes = [_I32, _I64, _P, _P]
            getattr(L, f"hsgo_heat_bath_draw_{suf}").argtypes = [_P, real, real, real, _P]
            getattr(L, f"hsgo_elem_consts_{suf}").argtypes = [_P, _P, _P]
            fn = getattr(L, f"hsgo_sweep_{suf}")
            fn.argtypes = [_I32, _U64, _U64, _I32, _D, _I32, _I32, _I32, _I32, _P, _P, _P, _D,
                           _P, _P, _P]
            fn.restype = ctypes.c_int
            getattr(L, f"hsgo_energy_{suf}").argtypes = [_I32, _P, _P]
            getattr(L, f"hsgo_energy_{suf}").restype = _D
            getattr(L, f"hsgo_overlap_{suf}").argtypes = [_I32, _P, _P, _P]
            getattr(L, f"hsgo_renormalise_{suf}").argtypes = [_I64, _P]
        _lib = L
    return _lib


def _suf(dtype) -> str:
    dt = np.dtype(dtype)
    if dt == np.float32:
        return "f32"
    if dt == np.float64:
        return "f64"
    raise TypeError(f"oracle computes in float32 or float64, not {dt}")


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _key(seed: int) -> np.ndarray:
    return np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)


def threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(lib().hsgo_threads())


def set_threads(n: int) -> None:
    lib().hsgo_set_threads(int(n))


# ----------------------------------------------------------------------------- RNG
def philox(ctr, seed: int) -> np.ndarray:
    """Philox4x32-10 blocks for counters ``ctr`` (shape (n, 4)) and key ``seed``."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(-1, 4))
    out = np.empty_like(c)
    lib().hsgo_philox_many(c.shape[0], _ptr(c), _ptr(_key(seed)), _ptr(out))
    return out


def u01(w) -> np.ndarray:
    """The exact uniforms ``(2*(w >> 9) + 1) * 2**-24`` as float64."""
    w = np.ascontiguousarray(np.asarray(w, dtype=np.uint32).ravel())
    out = np.empty(w.shape, dtype=np.float64)
    lib().hsgo_u01_many(w.size, _ptr(w), _ptr(out))
    return out


def poly_coefs(dtype) -> np.ndarray:
    out = np.empty(18, dtype=np.dtype(dtype))
    getattr(lib(), f"hsgo_poly_coefs_{_suf(dtype)}")(_ptr(out))
    return out


def sincos_2pi(u: float, dtype=np.float64):
    suf = _suf(dtype)
    s = np.zeros(1, dtype=dtype)
    c = np.zeros(1, dtype=dtype)
    getattr(lib(), f"hsgo_sincos_2pi_{suf}")(float(np.dtype(dtype).type(u)), _ptr(s), _ptr(c))
    return s[0], c[0]


_ELEM = {"exp": 0, "expm1": 1, "log": 2, "log1p": 3}


def elem(name: str, x, dtype=np.float64) -> np.ndarray:
    """The oracle's own exp / expm1 (x in [x_min, 0]), log (x > 0, normal) or log1p
    (|x| <= 1/2), element-wise in the given precision."""
    a = np.ascontiguousarray(np.asarray(x, dtype=dtype).ravel())
    out = np.empty_like(a)
    getattr(lib(), f"hsgo_elem_many_{_suf(dtype)}")(_ELEM[name], a.size, _ptr(a), _ptr(out))
    return out


def elem_consts(dtype):
    """(1/n! for n < 18, 1/(2j+1) for j < 18, [ln2 head, ln2 tail, log2 e, sqrt(1/2)])."""
    e = np.empty(18, dtype=dtype)
    a = np.empty(18, dtype=dtype)
    l = np.empty(4, dtype=dtype)
    getattr(lib(), f"hsgo_elem_consts_{_suf(dtype)}")(_ptr(e), _ptr(a), _ptr(l))
    return e, a, l


def heat_bath_draw(h, beta: float, u0: float, u1: float, dtype=np.float64) -> np.ndarray:
    hh = np.ascontiguousarray(np.asarray(h, dtype=dtype))
    out = np.zeros(3, dtype=dtype)
    getattr(lib(), f"hsgo_heat_bath_draw_{_suf(dtype)}")(_ptr(hh), float(beta), float(u0),
                                                         float(u1), _ptr(out))
    return out


def trial_spin(u0: float, u1: float, dtype=np.float64) -> np.ndarray:
    out = np.zeros(3, dtype=dtype)
    getattr(lib(), f"hsgo_trial_spin_{_suf(dtype)}")(float(u0), float(u1), _ptr(out))
    return out


# --------------------------------------------------------------------------- state
def init(L: int, seed: int, dtype=np.float32):
    """Philox initial state: spins uniform on the sphere, couplings N(0,1)."""
    N = L ** 3
    spins = np.zeros((3, N), dtype=dtype)
    J = np.zeros((3, N), dtype=dtype)
    getattr(lib(), f"hsgo_init_{_suf(dtype)}")(L, seed, _ptr(spins), _ptr(J))
    return spins, J


def local_field(L: int, spins: np.ndarray, J: np.ndarray, x: int, y: int, z: int) -> np.ndarray:
    h = np.zeros(3, dtype=spins.dtype)
    getattr(lib(), f"hsgo_local_field_{_suf(spins.dtype)}")(
        L, _ptr(np.ascontiguousarray(spins)), _ptr(np.ascontiguousarray(J)), x, y, z, _ptr(h))
    return h


def field(Jn, nbs, dtype=np.float64) -> np.ndarray:
    """Local field from a site's six couplings Jn (+x, -x, +y, -y, +z, -z) and its six
    neighbours' spins nbs (shape (6, 3), same order), in the order of local_field."""
    jn = np.ascontiguousarray(np.asarray(Jn, dtype=dtype))
    nb = np.ascontiguousarray(np.asarray(nbs, dtype=dtype).reshape(18))
    h = np.zeros(3, dtype=dtype)
    getattr(lib(), f"hsgo_field_{_suf(dtype)}")(_ptr(jn), _ptr(nb), _ptr(h))
    return h


def site_update(mode: int, h, s, *, seed: int, sweep: int, site: int, phase: int, k: int,
                T: float, margin_eps: float = 1e-6, dtype=np.float64):
    """One site's update as the sweep makes it (mode 0 Metropolis, 1 over-relaxation,
    2 heat bath): returns (new spin, number of flagged decisions)."""
    hh = np.ascontiguousarray(np.asarray(h, dtype=dtype))
    out = np.array(s, dtype=dtype, copy=True)
    fl = getattr(lib(), f"hsgo_site_update_{_suf(dtype)}")(
        int(mode), _ptr(hh), _ptr(out), int(seed), int(sweep), int(site), int(phase), int(k),
        float(T), float(margin_eps), None, None)
    return out, int(fl)


def overrelax_site(h, s) -> np.ndarray:
    h = np.ascontiguousarray(h)
    out = np.array(s, dtype=h.dtype, copy=True)
    getattr(lib(), f"hsgo_overrelax_site_{_suf(h.dtype)}")(_ptr(h), _ptr(out))
    return out


def sweep(L: int, seed: int, spins: np.ndarray, J: np.ndarray, *, T: float, k: int = 1,
          n_or: int = 0, renorm_every: int = 0, n_sweeps: int = 1, sweep0: int = 0,
          E: float | None = None, heat_bath: bool = False, margin_eps: float = 1e-6,
          taint: np.ndarray | None = None) -> dict:
    """Run ``n_sweeps`` sweeps in place on ``spins`` (shape (3, N), C-contiguous).

    Returns ``{"E": tracked energy (E + accepted changes; None if E is None),
    "n_flagged": decisions within margin_eps of their threshold, "n_accepted": ...}``.
    ``taint`` (uint8, shape (N,)) is updated in place when given.
    """
    assert spins.flags.c_contiguous and J.flags.c_contiguous
    assert spins.dtype == J.dtype and spins.shape == (3, L ** 3) and J.shape == (3, L ** 3)
    e = np.array([0.0 if E is None else float(E)])
    nf = np.zeros(1, dtype=np.int64)
    na = np.zeros(1, dtype=np.int64)
    tp = None
    if taint is not None:
        assert taint.dtype == np.uint8 and taint.shape == (L ** 3,) and taint.flags.c_contiguous
        tp = _ptr(taint)
    rc = getattr(lib(), f"hsgo_sweep_{_suf(spins.dtype)}")(
        L, seed, sweep0, n_sweeps, float(T), k, n_or, renorm_every, int(bool(heat_bath)),
        _ptr(spins), _ptr(J), _ptr(e), margin_eps, tp, _ptr(nf), _ptr(na))
    if rc != 0:
        raise ValueError("oracle sweep rejected its arguments")
    return {"E": None if E is None else float(e[0]), "n_flagged": int(nf[0]),
            "n_accepted": int(na[0])}


def energy(L: int, spins: np.ndarray, J: np.ndarray) -> float:
    return float(getattr(lib(), f"hsgo_energy_{_suf(spins.dtype)}")(
        L, _ptr(np.ascontiguousarray(spins)), _ptr(np.ascontiguousarray(J))))


def overlap(L: int, a: np.ndarray, b: np.ndarray):
    """Returns (Q (3x3), m_a (3,), m_b (3,)) in float64."""
    out = np.zeros(15, dtype=np.float64)
    getattr(lib(), f"hsgo_overlap_{_suf(a.dtype)}")(
        L, _ptr(np.ascontiguousarray(a)), _ptr(np.ascontiguousarray(b)), _ptr(out))
    return out[:9].reshape(3, 3), out[9:12], out[12:15]


def renormalise(spins: np.ndarray) -> None:
    assert spins.flags.c_contiguous and spins.shape[0] == 3
    getattr(lib(), f"hsgo_renormalise_{_suf(spins.dtype)}")(spins.shape[1], _ptr(spins))


def pt_swap(beta_of_slot, E_of_chain, chain_at_slot: np.ndarray, seed: int, stream_id: int,
            round_: int, accepted_pairs: np.ndarray | None = None) -> int:
    """Replica-exchange round in place on ``chain_at_slot`` (int32)."""
    b = np.ascontiguousarray(beta_of_slot, dtype=np.float64)
    e = np.ascontiguousarray(E_of_chain, dtype=np.float64)
    assert chain_at_slot.dtype == np.int32 and chain_at_slot.flags.c_contiguous
    ap = None
    if accepted_pairs is not None:
        assert accepted_pairs.dtype == np.int32
        ap = _ptr(accepted_pairs)
    return int(lib().hsgo_pt_swap(b.size, _ptr(b), _ptr(e), _ptr(chain_at_slot), seed,
                                  stream_id, round_, ap))
