"""The allocation-free sweep (hsg_sweep_noalloc) against hsg_sweep: two calls in a row on
one GPU, the second on a smaller lattice (the library's scratch array keeps the first
call's contents and must be cleared), each compared with hsg_sweep on an identical
lattice: spins bit for bit, the sweep index exactly, the tracked energy up to nothing
(the same kernels add the same partials in the same order)."""
from __future__ import annotations

import ctypes

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hsg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1006_2566_amd as m
    m.lib()
    return m


def noalloc_sweep(hsg, lat, *, T, k, n_or, R, n, flags):
    """hsg_sweep_noalloc on the lattice's buffers, its descriptor stripped of the work
    buffer."""
    d = hsg._Lattice(lat._d.L, lat._d.dtype, lat._d.seed, lat._d.sweep, lat._d.spins,
                     lat._d.J, lat._d.E, None, 0)
    p = hsg._SweepParams(float(T), int(k), int(n_or), int(R), int(flags))
    hsg.check(hsg.lib().hsg_sweep_noalloc(ctypes.byref(d), ctypes.byref(p), int(n),
                                          hsg._stream(None)))
    lat._d.sweep = d.sweep


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_sweep_equals_sweep(hsg, dtype):
    hsg.lib().hsg_sweep_noalloc.argtypes = [ctypes.POINTER(hsg._Lattice),
                                            ctypes.POINTER(hsg._SweepParams), ctypes.c_int32,
                                            ctypes.c_void_p]
    cases = [  # L, k, n_or, R, n sweeps, heat bath, flags
        (96, 4, 1, 3, 5, False, hsg.HSG_SNAKE),
        (24, 1, 2, 2, 3, True, 0),  # smaller: the first call's partials must not leak in
    ]
    for L, k, n_or, R, n, hb, flags in cases:
        f = flags | (hsg.HSG_HEAT_BATH if hb else 0)
        ref = hsg.Lattice(L, dtype, seed=31 + L)
        got = hsg.Lattice(L, dtype, seed=31 + L)
        ref.sweep_index = got.sweep_index = 4
        ref.sweep(T=0.45, k=k, n_or=n_or, renorm_every=R, n_sweeps=n, flags=f)
        noalloc_sweep(hsg, got, T=0.45, k=k, n_or=n_or, R=R, n=n, flags=f)
        torch.cuda.synchronize()
        same = bool(torch.equal(ref.spins, got.spins))
        Er, Eg = ref.energy().item(), got.energy().item()
        print(f"[noalloc] L={L} {dtype} k={k} n_or={n_or} hb={hb}: bitwise={same} "
              f"E={Er:.9f} dE={Eg - Er:.3e}", flush=True)
        assert same
        assert got.sweep_index == ref.sweep_index == 4 + n
        assert Eg == Er
        Erec = got.energy(recompute=True).item()
        assert abs(Eg - Erec) <= (1e-5 if dtype == torch.float32 else 1e-12) * abs(Erec)
