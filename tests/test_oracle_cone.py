"""Pins for the one-by-one recomputation of sampled sites (tests/cone.py), which checks the
GPU at lattice sizes the whole-lattice oracle cannot run: on small lattices it must
reproduce the oracle's sweep bit for bit at every site, and its taint flags the oracle's
taint map exactly."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from tests import cone, inputs


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("L,k,n_or,n,R,T,hb", [
    (6, 4, 1, 2, 1, 0.3, False),   # Metropolis, over-relaxation, renormalisation inside
    (8, 1, 2, 1, 0, 0.5, False),
    (6, 3, 0, 3, 2, 1.0, True),    # heat bath
    (4, 0, 2, 2, 0, 0.4, False),   # over-relaxation only
])
def test_cone_reproduces_the_sweep(dtype, L, k, n_or, n, R, T, hb):
    seed, sweep0 = 23, 4
    spins, J = inputs.random_state(L, 11, dtype)
    ref = spins.copy()
    taint = np.zeros(L ** 3, dtype=np.uint8)
    O.sweep(L, seed, ref, J, T=T, k=k, n_or=n_or, renorm_every=R, n_sweeps=n, sweep0=sweep0,
            heat_bath=hb, taint=taint)
    steps = cone.schedule(k, n_or, n, sweep0=sweep0, heat_bath=hb, renorm_every=R)
    sites = np.arange(L ** 3)
    c = cone.Cone(L, dtype, seed=seed, T=T, k=k, steps=steps, sites=sites, spins0=spins, J=J)
    for i in range(L ** 3):
        s, t = c.value(i)
        np.testing.assert_array_equal(s, ref[:, i])
        assert t == bool(taint[i]), i


def test_cone_flags_follow_flagged_decisions():
    """With a margin wide enough that a fair share of decisions is flagged, the cone's
    flags equal the oracle's taint map site by site."""
    L, seed, T, k = 6, 3, 0.4, 2
    spins, J = inputs.random_state(L, 5, np.float64)
    ref = spins.copy()
    taint = np.zeros(L ** 3, dtype=np.uint8)
    r = O.sweep(L, seed, ref, J, T=T, k=k, n_or=1, n_sweeps=1, margin_eps=0.05, taint=taint)
    assert r["n_flagged"] > 0 and 0 < taint.sum() < L ** 3
    c = cone.Cone(L, np.float64, seed=seed, T=T, k=k, steps=cone.schedule(k, 1, 1),
                  sites=np.arange(L ** 3), spins0=spins, J=J, margin_eps=0.05)
    flags = np.array([c.value(i)[1] for i in range(L ** 3)])
    np.testing.assert_array_equal(flags, taint.astype(bool))


def test_within_counts_the_l1_ball():
    """Sites within r steps on a large periodic lattice: the L1 ball,
    (2r + 1)(2r^2 + 2r + 3)/3 sites."""
    for r in range(5):
        got = len(cone.within(64, [cone.index(64, 10, 20, 30)], r))
        assert got == (2 * r + 1) * (2 * r * r + 2 * r + 3) // 3
