"""Pins for the oracle's bookkeeping of near-threshold Metropolis decisions.

A decision is "flagged" when its uniform u lies within margin_eps of the acceptance
probability min(1, exp(-beta dE)); its site, and every site later updated next to a
flagged or tainted site in the same call (the causal cone), is "tainted".  The GPU
parity tests leave tainted sites out, so the count and the cone must be right.

The replay below recomputes every decision independently of the oracle's colour
pass: the per-site field and the trial point come from the oracle's pinned
building blocks (local field, trial spin, Philox, uniforms), every other operation
is spelled out here with the C library's fmaf / fma / expf / exp through ctypes (the
primitives the oracle's C code calls) and numpy's IEEE scalar arithmetic, and the
cone is propagated over the whole lattice with periodic rolls.  The replay must
give the oracle's spins bit for bit, its flag count exactly and its taint map
exactly.
"""
from __future__ import annotations

import ctypes
import ctypes.util

import numpy as np
import pytest

import oracle as O
from tests import inputs

F32, F64 = np.float32, np.float64

_libm = ctypes.CDLL(ctypes.util.find_library("m") or "libm.so.6")
_libm.fmaf.argtypes = [ctypes.c_float] * 3
_libm.fmaf.restype = ctypes.c_float
_libm.fma.argtypes = [ctypes.c_double] * 3
_libm.fma.restype = ctypes.c_double
_libm.expf.argtypes = [ctypes.c_float]
_libm.expf.restype = ctypes.c_float
_libm.exp.argtypes = [ctypes.c_double]
_libm.exp.restype = ctypes.c_double


def _fma(dt, a, b, c):
    f = _libm.fmaf if dt == F32 else _libm.fma
    return dt(f(float(a), float(b), float(c)))


def _exp(dt, x):
    return dt((_libm.expf if dt == F32 else _libm.exp)(float(x)))


def _dot3(dt, a, b):
    acc = dt(a[0]) * dt(b[0])
    acc = _fma(dt, a[1], b[1], acc)
    return _fma(dt, a[2], b[2], acc)


def _uniforms(L, seed, sweep, site, phase, n):
    """The first n Monte Carlo uniforms of a site in a phase: words of the Philox
    blocks with counter (sweep, site, (phase << 16) | block, tag 0), in order."""
    nb = (n + 3) // 4
    ctr = np.array([[sweep, site, (phase << 16) | b, O.TAG_MH] for b in range(nb)],
                   dtype=np.uint32)
    return O.u01(O.philox(ctr, seed).ravel())[:n]


def _neighbour_or(L, t):
    """OR over the six periodic neighbours of every site of a canonical (N,) map."""
    g = t.reshape(L, L, L).astype(bool)  # [z, y, x]
    out = np.zeros_like(g)
    for ax in range(3):
        out |= np.roll(g, 1, axis=ax) | np.roll(g, -1, axis=ax)
    return out.reshape(-1)


def replay(L, seed, spins, J, *, T, k, n_or, sweep0, n_sweeps, margin_eps,
           clamp_p=True):
    """Independent replay of n_sweeps sweeps (Metropolis phase of k hits, then n_or
    over-relaxation phases; colour 0 then colour 1 in each).  Returns the final spins,
    the number of flagged decisions and the taint map.  clamp_p=False measures the
    margin against the raw exp(-beta dE) instead (the sensitivity check only)."""
    dt = spins.dtype.type
    s = spins.copy()
    N = L ** 3
    beta = dt(1.0 / T)
    col = inputs.colours(L)
    taint = np.zeros(N, dtype=bool)
    n_flag = 0
    coords = [(i % L, (i // L) % L, i // (L * L)) for i in range(N)]
    for n in range(n_sweeps):
        sweep = sweep0 + n
        for phase in range(0, n_or + 1):
            if phase == 0 and k == 0:
                continue
            for c in (0, 1):
                flag = np.zeros(N, dtype=bool)
                sites = np.nonzero(col == c)[0]
                new = {}
                for i in sites:
                    x, y, z = coords[i]
                    h = O.local_field(L, s, J, x, y, z)
                    cur = s[:, i].copy()
                    if phase > 0:
                        new[i] = O.overrelax_site(h, cur)
                        continue
                    sh = _dot3(dt, cur, h)
                    u = _uniforms(L, seed, sweep, i, phase, 3 * k)
                    for j in range(k):
                        t = O.trial_spin(u[3 * j], u[3 * j + 1], dt)
                        th = _dot3(dt, t, h)
                        dE = dt(sh - th)
                        p = _exp(dt, dt(-beta) * dE)
                        u2 = dt(u[3 * j + 2])
                        pm = (float(p) if p < 1 else 1.0) if clamp_p else float(p)
                        if abs(float(u2) - pm) < margin_eps:
                            n_flag += 1
                            flag[i] = True
                        if dE <= 0 or u2 < p:
                            cur, sh = t, th
                    new[i] = cur
                for i, v in new.items():
                    s[:, i] = v
                # the cone: a site of this colour is tainted if it was, if a neighbour
                # (all of the other colour) is, or if one of its decisions was flagged
                upd = col == c
                taint = np.where(upd, taint | _neighbour_or(L, taint) | flag, taint)
    return s, n_flag, taint


CASES = [
    # L, dtype, state, T, k, n_or, n_sweeps, margin_eps
    (4, F32, "random", 0.5, 4, 0, 2, 0.05),
    (4, F64, "random", 0.5, 4, 1, 2, 0.05),
    (6, F32, "random", 1.0, 1, 1, 2, 0.02),
    (6, F32, "frozen", 0.7, 4, 0, 1, 0.1),
    (6, F64, "frozen", 0.3, 2, 0, 2, 0.2),
    (4, F32, "random", 0.2, 8, 0, 1, 1e-6),
    (2, F32, "random", 1.0, 3, 1, 3, 0.05),
    (8, F32, "random", 0.5, 4, 0, 1, 2e-3),   # a few flags, a partial cone
    (8, F64, "random", 0.3, 4, 1, 1, 2e-3),
]


@pytest.mark.parametrize("L,dtype,state,T,k,n_or,n_sweeps,eps", CASES)
def test_flag_count_and_taint_cone(L, dtype, state, T, k, n_or, n_sweeps, eps):
    gen = inputs.random_state if state == "random" else inputs.frozen_field_state
    spins, J = gen(L, 31 + L, dtype)
    seed, sweep0 = 900 + L, 3
    ref_s, ref_n, ref_t = replay(L, seed, spins, J, T=T, k=k, n_or=n_or, sweep0=sweep0,
                                 n_sweeps=n_sweeps, margin_eps=eps)
    got = spins.copy()
    taint = np.zeros(L ** 3, dtype=np.uint8)
    r = O.sweep(L, seed, got, J, T=T, k=k, n_or=n_or, n_sweeps=n_sweeps, sweep0=sweep0,
                margin_eps=eps, taint=taint)
    np.testing.assert_array_equal(got, ref_s)
    assert r["n_flagged"] == ref_n
    np.testing.assert_array_equal(taint.astype(bool), ref_t)
    if eps > 1e-6:
        # the widened bands make flags common: the check has something to count
        assert ref_n > 0 and ref_t.any()
    if L == 8:
        # one sweep from a few flags: the cone is a proper subset of the lattice
        assert 0 < ref_t.sum() < L ** 3 // 2


def test_flag_rule_is_sensitive_to_the_clamp():
    """The flag band is around min(1, p): counting |u - p| with the raw p (a
    plausible slip) gives a different count on these inputs, so the exact-count pin
    above would catch it."""
    L, dtype = 6, F32
    spins, J = inputs.random_state(L, 5, dtype)
    kw = dict(T=0.5, k=4, n_or=0, sweep0=0, n_sweeps=1, margin_eps=0.1)
    _, n_clamped, t_clamped = replay(L, 17, spins, J, **kw)
    _, n_raw, t_raw = replay(L, 17, spins, J, clamp_p=False, **kw)
    assert n_clamped != n_raw
    got = spins.copy()
    taint = np.zeros(L ** 3, dtype=np.uint8)
    r = O.sweep(L, 17, got, J, margin_eps=0.1, taint=taint, **{k: v for k, v in kw.items()
                                                                if k != "margin_eps"})
    assert r["n_flagged"] == n_clamped != n_raw


@pytest.mark.parametrize("dtype", [F32, F64])
def test_tie_rejects_and_is_flagged(dtype):
    """A decision with u exactly equal to exp(-beta dE) rejects (accept iff u < p)
    and is flagged.  Site 0 of an L = 2 lattice is turned along its field, so its one
    trial cannot lower the energy (dE > 0); beta is then searched, one ulp at a time,
    for the value at which the library exp returns the site's uniform exactly."""
    L, seed, sweep = 2, 4242, 0
    dt = np.dtype(dtype).type
    spins, J = inputs.random_state(L, 8, dtype)
    h = O.local_field(L, spins, J, 0, 0, 0)
    spins[:, 0] = (h / np.sqrt(float(_dot3(dt, h, h)))).astype(dtype)
    sh = _dot3(dt, spins[:, 0], h)
    found = None
    for s_try in range(200):
        u = _uniforms(L, seed, sweep + s_try, 0, 0, 3)
        t = O.trial_spin(u[0], u[1], dtype)
        dE = dt(sh - _dot3(dt, t, h))
        u2 = dt(u[2])
        if not (dE > 0 and 0.05 < u2 < 0.95):
            continue
        b = dt(-np.log(float(u2)) / float(dE))
        cands, up, dn = [b], b, b
        for _ in range(4000):
            up, dn = np.nextafter(up, dt(np.inf)), np.nextafter(dn, dt(0))
            cands += [up, dn]
        for cand in cands:
            if _exp(dt, dt(-cand) * dE) == u2:
                found = (s_try, cand)
                break
        if found:
            break
    if found is None:
        pytest.skip("no exact tie reachable for these draws")
    s_try, beta = found
    T = 1.0 / float(beta)
    assert dt(1.0 / T) == beta
    before = spins.copy()
    taint = np.zeros(L ** 3, dtype=np.uint8)
    r = O.sweep(L, seed, spins, J, T=T, k=1, n_or=0, n_sweeps=1, sweep0=sweep + s_try,
                taint=taint)
    np.testing.assert_array_equal(spins[:, 0], before[:, 0])  # rejected
    assert taint[0] == 1 and r["n_flagged"] >= 1
