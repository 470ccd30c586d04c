"""Seeded synthetic inputs shared by the oracle and the GPU library in tests.

This module only draws inputs (numpy's PCG64 generator); it holds none of the
sweep's arithmetic.  Shapes follow the canonical layout: spins and couplings are
(3, N) arrays with site index i = x + L*y + L*L*z.
"""
from __future__ import annotations

import numpy as np


def random_state(L: int, seed: int, dtype=np.float32):
    """Spins uniform on the unit sphere (normalised Gaussian triples, rounded to
    dtype) and couplings N(0,1) on the 3*L^3 bonds."""
    rng = np.random.default_rng(seed)
    N = L ** 3
    g = rng.standard_normal((3, N))
    spins = (g / np.linalg.norm(g, axis=0)).astype(dtype)
    J = rng.standard_normal((3, N)).astype(dtype)
    return np.ascontiguousarray(spins), np.ascontiguousarray(J)


def colours(L: int) -> np.ndarray:
    x, y, z = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    # canonical order: i = x + L*y + L*L*z  ->  reshape with z slowest
    c = (x + y + z) & 1
    return np.ascontiguousarray(c.transpose(2, 1, 0).reshape(-1)).astype(np.int64)


def frozen_field_state(L: int, seed: int, dtype=np.float32):
    """All couplings +1, colour-1 spins along +z, colour-0 spins random: every
    colour-0 site then sees the field (0, 0, 6) during the first colour pass."""
    spins, _ = random_state(L, seed, dtype)
    c = colours(L)
    spins[:, c == 1] = np.array([[0.0], [0.0], [1.0]], dtype=dtype)
    J = np.ones((3, L ** 3), dtype=dtype)
    return np.ascontiguousarray(spins), J


