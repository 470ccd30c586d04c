"""Host-side estimators of the package (chi_SG, xi, Binder cumulant over a series of
Fourier-overlap records) against the oracle's definitions, on synthetic record
series; no GPU involved."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import observables as OB


def synthetic_records(rng, n_meas, shape):
    """Record series with random q2(0) and q2(k_min) columns (the estimators read only
    those two)."""
    r = np.zeros((n_meas,) + shape + (65,))
    r[..., 63] = rng.gamma(4.5, 0.002, size=(n_meas,) + shape)
    r[..., 64] = r[..., 63] * rng.uniform(0.2, 0.9, size=(n_meas,) + shape)
    return r


def test_moments_and_estimators_match_oracle():
    from paper_1006_2566_amd import observables as M
    rng = np.random.default_rng(3)
    n_pairs, n_temps, L = 5, 4, 16
    rec = synthetic_records(rng, 30, (n_pairs, n_temps))
    mom = M.OverlapMoments((n_pairs, n_temps))
    for r in rec:
        mom.add(r)
    est = M.by_size(mom, [L] * n_pairs)[L]
    for t in range(n_temps):
        # the oracle's estimators over the pooled series of one temperature: pooling
        # equal-length series is the mean over pairs of the thermal means
        pooled = rec[:, :, t, :].reshape(-1, 65)
        chi0, chik = OB.chi_sg(pooled, L ** 3)
        assert est["chi0"][t] == pytest.approx(chi0, rel=1e-12)
        assert est["chik"][t] == pytest.approx(chik, rel=1e-12)
        assert est["xi"][t] == pytest.approx(OB.xi_second_moment(chi0, chik, L), rel=1e-12)
        assert est["g"][t] == pytest.approx(OB.binder_g(pooled), rel=1e-12, abs=1e-12)


def test_by_size_separates_lattice_sizes():
    from paper_1006_2566_amd import observables as M
    rng = np.random.default_rng(4)
    Ls = [8, 12, 8, 12, 12]
    rec = synthetic_records(rng, 10, (len(Ls), 2))
    mom = M.OverlapMoments((len(Ls), 2))
    for r in rec:
        mom.add(r)
    out = M.by_size(mom, Ls)
    assert sorted(out) == [8, 12]
    sel = rec[:, [1, 3, 4], 0, :].reshape(-1, 65)
    assert out[12]["chi0"][0] == pytest.approx(OB.chi_sg(sel, 12 ** 3)[0], rel=1e-12)


def test_moments_need_a_measurement():
    from paper_1006_2566_amd import observables as M
    with pytest.raises(ValueError):
        M.OverlapMoments((2,)).thermal()
