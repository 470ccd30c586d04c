"""Degenerate calls through the C ABI: a call of zero sweeps leaves spins, tracked energy
and sweep index untouched under every traversal (and records no launch, or clears nothing
it should not, in the timed and allocation-free entry points); every traversal flag on
the smallest lattices, where the LDS launches do not apply, gives the plain schedule's
spins bit for bit."""
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


def traversals(m):
    return {"GM": 0, "GM+S": m.HSG_SNAKE, "PH": m.HSG_SNAKE | m.HSG_PHASE_LAUNCH,
            "PH+MC": m.HSG_SNAKE | m.HSG_PHASE_MC, "SM4P": m.HSG_FUSED,
            "CA": m.HSG_PLANE_LAUNCH, "TEXT": m.HSG_SNAKE | m.HSG_STREAM_LOADS}


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_zero_sweeps_change_nothing(hsg, dtype):
    L = 64
    lat = hsg.Lattice(L, dtype, seed=3)
    lat.sweep(T=0.5, k=2, n_or=1, n_sweeps=2)  # a state that is not the initial one
    torch.cuda.synchronize()
    spins, E, idx = lat.spins.clone(), lat.E.clone(), lat.sweep_index
    for name, flags in traversals(hsg).items():
        lat.sweep(T=0.5, k=4, n_or=1, renorm_every=1, n_sweeps=0, flags=flags)
        assert lat.sweep_timed(T=0.5, k=4, n_or=1, n_sweeps=0, flags=flags) == [], name
        torch.cuda.synchronize()
        assert torch.equal(lat.spins, spins), name
        assert torch.equal(lat.E, E), name
        assert lat.sweep_index == idx, name
    d = hsg._Lattice(lat._d.L, lat._d.dtype, lat._d.seed, lat._d.sweep, lat._d.spins,
                     lat._d.J, lat._d.E, None, 0)
    p = hsg._SweepParams(0.5, 4, 1, 1, int(hsg.HSG_SNAKE))
    hsg.check(hsg.lib().hsg_sweep_noalloc(ctypes.byref(d), ctypes.byref(p), 0,
                                          hsg._stream(None)))
    torch.cuda.synchronize()
    assert torch.equal(lat.spins, spins) and torch.equal(lat.E, E) and d.sweep == idx


@pytest.mark.parametrize("L", [2, 4, 6])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_every_traversal_on_the_smallest_lattices(hsg, L, dtype):
    runs = {}
    for name, flags in traversals(hsg).items():
        lat = hsg.Lattice(L, dtype, seed=11)
        lat.sweep(T=0.7, k=3, n_or=2, renorm_every=2, n_sweeps=3, flags=flags)
        runs[name] = (lat.spins.clone(), lat.energy().item())
    ref_s, ref_E = runs["GM"]
    for name, (s, E) in runs.items():
        assert torch.equal(s, ref_s), name
        assert E == ref_E, name
