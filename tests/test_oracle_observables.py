"""Pins for the oracle's spin-glass observables (Fourier components of the tensor
overlap, chi_SG, the second-moment correlation length, the Binder cumulant): each
checked against a fact fixed outside the oracle -- a brute-force sum over explicit
site coordinates, closed forms for uniform and plane-wave states, translation
covariance, the C oracle's k = 0 overlap, the exact mean of uncorrelated replicas,
and the moment ratios of constant and Gaussian order parameters."""
from __future__ import annotations

import cmath
import math

import numpy as np
import pytest

import oracle as O
from oracle import observables as OB
from tests import inputs


def brute_record(L, a, b):
    """The record by explicit loops over sites and their coordinates."""
    N = L ** 3
    Q0 = [0.0] * 9
    Qk = [[0j] * 9 for _ in range(3)]
    for i in range(N):
        x, y, z = i % L, (i // L) % L, i // (L * L)
        for mu in range(3):
            for nu in range(3):
                q = float(a[mu, i]) * float(b[nu, i])
                Q0[3 * mu + nu] += q / N
                for d, r in enumerate((x, y, z)):
                    Qk[d][3 * mu + nu] += q * cmath.exp(2j * math.pi * r / L) / N
    out = np.zeros(65)
    out[:9] = Q0
    for d in range(3):
        out[9 + 18 * d:18 + 18 * d] = [v.real for v in Qk[d]]
        out[18 + 18 * d:27 + 18 * d] = [v.imag for v in Qk[d]]
    out[63] = sum(v * v for v in Q0)
    out[64] = sum(abs(v) ** 2 for row in Qk for v in row) / 3
    return out


def coords(L):
    i = np.arange(L ** 3)
    return i % L, (i // L) % L, i // (L * L)


@pytest.mark.parametrize("L", [2, 3, 4])
def test_record_matches_brute_force(L):
    a, _ = inputs.random_state(L, 11, np.float64)
    b, _ = inputs.random_state(L, 12, np.float64)
    np.testing.assert_allclose(OB.overlap_fourier(L, a, b), brute_record(L, a, b), rtol=0,
                               atol=1e-14)


def test_k0_block_equals_c_oracle_overlap():
    L = 8
    a, _ = inputs.random_state(L, 3, np.float64)
    b, _ = inputs.random_state(L, 4, np.float64)
    Q, _, _ = O.overlap(L, a, b)
    np.testing.assert_allclose(OB.overlap_fourier(L, a, b)[:9], Q.reshape(-1), rtol=0,
                               atol=1e-15)


def test_uniform_state():
    """a = u, b = v everywhere: Q(0) = u v^T and every k != 0 component vanishes."""
    L = 6
    u = np.array([0.6, 0.0, 0.8])
    v = np.array([0.0, -1.0, 0.0])
    a = np.repeat(u[:, None], L ** 3, axis=1)
    b = np.repeat(v[:, None], L ** 3, axis=1)
    r = OB.overlap_fourier(L, a, b)
    np.testing.assert_allclose(r[:9], np.outer(u, v).reshape(-1), atol=1e-15)
    np.testing.assert_allclose(r[9:63], 0.0, atol=1e-15)
    assert r[63] == pytest.approx(1.0, abs=1e-15) and r[64] == pytest.approx(0.0, abs=1e-30)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_plane_wave(d):
    """a_r = (cos t, sin t, 0), t = 2 pi r_d / L, b = e_x: q^{00} = cos t, q^{10} = sin t,
    so Q^{00}(k_d) = 1/2, Q^{10}(k_d) = i/2 (sign of the exponent), nothing along the
    other axes and nothing at k = 0."""
    L = 8
    t = 2 * np.pi * coords(L)[d] / L
    a = np.stack([np.cos(t), np.sin(t), np.zeros_like(t)])
    b = np.zeros_like(a)
    b[0] = 1.0
    r = OB.overlap_fourier(L, a, b)
    want = np.zeros(65)
    want[9 + 18 * d + 0] = 0.5      # Re Q^{00}(k_d)
    want[18 + 18 * d + 3] = 0.5     # Im Q^{10}(k_d)
    want[64] = (0.25 + 0.25) / 3
    np.testing.assert_allclose(r, want, atol=1e-15)


def test_plane_wave_self_overlap():
    """b = a = (cos t, sin t, 0): Q(0) = diag(1/2, 1/2, 0); cos^2 and sin cos hold only
    the harmonics 0 and 2, so every k_min component vanishes (L = 8)."""
    L = 8
    t = 2 * np.pi * coords(L)[1] / L
    a = np.stack([np.cos(t), np.sin(t), np.zeros_like(t)])
    r = OB.overlap_fourier(L, a, a)
    np.testing.assert_allclose(r[:9], [0.5, 0, 0, 0, 0.5, 0, 0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(r[9:63], 0.0, atol=1e-15)
    assert r[63] == pytest.approx(0.5, abs=1e-15)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_translation_multiplies_by_phase(d):
    """Shifting both configurations by +1 along d multiplies Q(k_d) by exp(+2 pi i / L)
    and leaves Q(0) and every |Q(k)| as they were."""
    L = 6
    a, _ = inputs.random_state(L, 5, np.float64)
    b, _ = inputs.random_state(L, 6, np.float64)
    axis = 3 - d  # (3, z, y, x) view
    sa = np.roll(a.reshape(3, L, L, L), 1, axis=axis).reshape(3, -1)
    sb = np.roll(b.reshape(3, L, L, L), 1, axis=axis).reshape(3, -1)
    r, s = OB.overlap_fourier(L, a, b), OB.overlap_fourier(L, sa, sb)
    np.testing.assert_allclose(s[:9], r[:9], atol=1e-15)
    for e in range(3):
        Qr = r[9 + 18 * e:18 + 18 * e] + 1j * r[18 + 18 * e:27 + 18 * e]
        Qs = s[9 + 18 * e:18 + 18 * e] + 1j * s[18 + 18 * e:27 + 18 * e]
        phase = np.exp(2j * np.pi / L) if e == d else 1.0
        np.testing.assert_allclose(Qs, phase * Qr, atol=1e-15)
    assert s[63] == pytest.approx(r[63], rel=1e-13) and s[64] == pytest.approx(r[64], rel=1e-13)


def test_uncorrelated_replicas_have_unit_chi():
    """Independent uniform spins: E[(a^mu b^nu)^2] = 1/9, so E[N q2(k)] = 1 at every k
    and chi(0) = chi(k_min) = 1 up to sampling noise (about 0.03 here)."""
    L, n = 6, 200
    rec = []
    for s in range(n):
        a, _ = inputs.random_state(L, 1000 + s, np.float64)
        b, _ = inputs.random_state(L, 5000 + s, np.float64)
        rec.append(OB.overlap_fourier(L, a, b))
    chi0, chik = OB.chi_sg(np.array(rec), L ** 3)
    assert abs(chi0 - 1.0) < 0.15 and abs(chik - 1.0) < 0.15


def test_xi_inverts_ornstein_zernike():
    """chi(k) = chi(0) / (1 + xi^2 khat^2), khat = 2 sin(k/2): the estimator returns xi."""
    L, xi = 16, 3.25
    khat2 = (2 * math.sin(math.pi / L)) ** 2
    chi0 = 40.0
    assert OB.xi_second_moment(chi0, chi0 / (1 + xi * xi * khat2), L) == pytest.approx(xi,
                                                                                     rel=1e-13)
    assert OB.xi_second_moment(chi0, chi0, L) == 0.0
    assert math.isnan(OB.xi_second_moment(1.0, 2.0, L))


def test_binder_limits():
    """g = 1 for a frozen order parameter; g = 0 when the 9 components are independent
    Gaussians (q2 ~ chi-square with 9 degrees: <q2^2>/<q2>^2 = 11/9)."""
    rec = np.zeros((50, 65))
    rec[:, 63] = 0.37
    assert OB.binder_g(rec) == pytest.approx(1.0, abs=1e-14)
    rng = np.random.default_rng(9)
    comp = rng.standard_normal((400000, 9)) * 0.1
    rec = np.zeros((comp.shape[0], 65))
    rec[:, 63] = (comp ** 2).sum(axis=1)
    assert abs(OB.binder_g(rec)) < 0.02
