"""Sampled sites of a run of sweeps recomputed one by one with the oracle's per-site
functions (test infrastructure).

Within a colour pass a site's new spin depends only on its own spin and its six
neighbours' spins before the pass: the neighbours have the other colour (§4), and the
draws are keyed by (seed, sweep, site, phase).  So a site's spin after P passes is fixed
by the spins within distance P of it before them.  `Cone` evaluates that dependency from
the initial state gathered at those sites: lattices too large for the oracle's
whole-lattice sweep (or for the host's memory) are checked on sampled sites.  The flag
a site carries says whether any Metropolis decision its value depends on lies within the
oracle's margin of its threshold (the oracle's taint, computed the other way round).
"""
from __future__ import annotations

import numpy as np

import oracle as O


def schedule(k: int, n_or: int, n_sweeps: int, *, sweep0: int = 0, heat_bath: bool = False,
             renorm_every: int = 0) -> list[tuple]:
    """The passes (and renormalisations) of n_sweeps sweeps in the oracle's order:
    ("pass", sweep, mode, colour, phase) and ("renorm",)."""
    out = []
    for sw in range(sweep0, sweep0 + n_sweeps):
        for phase in range(n_or + 1):
            if phase == 0 and k == 0:
                continue
            mode = 1 if phase > 0 else (2 if heat_bath else 0)
            for colour in (0, 1):
                out.append(("pass", sw, mode, colour, phase))
        if renorm_every > 0 and (sw + 1) % renorm_every == 0:
            out.append(("renorm",))
    return out


def coords(L: int, i: int) -> tuple[int, int, int]:
    return i % L, (i // L) % L, i // (L * L)


def index(L: int, x: int, y: int, z: int) -> int:
    return (x % L) + L * ((y % L) + L * (z % L))


def neighbours(L: int, i: int) -> list[int]:
    """+x, -x, +y, -y, +z, -z."""
    x, y, z = coords(L, i)
    return [index(L, x + 1, y, z), index(L, x - 1, y, z), index(L, x, y + 1, z),
            index(L, x, y - 1, z), index(L, x, y, z + 1), index(L, x, y, z - 1)]


def within(L: int, targets, radius: int) -> np.ndarray:
    """Sorted canonical indices of every site within `radius` steps of a target."""
    seen = set(int(t) for t in targets)
    front = set(seen)
    for _ in range(radius):
        nxt = set()
        for i in front:
            for j in neighbours(L, i):
                if j not in seen:
                    seen.add(j)
                    nxt.add(j)
        front = nxt
    return np.array(sorted(seen), dtype=np.int64)


class Cone:
    """Spin of a site after the first p steps of `steps`, from the initial spins and
    couplings given at the sites `sites` (arrays of shape (3, len(sites)), canonical
    couplings: component d is the +d bond stored at the site)."""

    def __init__(self, L: int, dtype, *, seed: int, T: float, k: int, steps: list[tuple],
                 sites: np.ndarray, spins0: np.ndarray, J: np.ndarray,
                 margin_eps: float = 1e-6):
        self.L, self.dtype, self.seed, self.T, self.k = L, np.dtype(dtype).type, seed, T, k
        self.margin_eps = margin_eps
        self.steps = steps
        self.pos = {int(s): n for n, s in enumerate(sites)}
        self.s0 = np.asarray(spins0, dtype=dtype)
        self.J = np.asarray(J, dtype=dtype)
        self.memo: dict[tuple[int, int], tuple[np.ndarray, bool]] = {}

    def _spin0(self, i: int) -> np.ndarray:
        return self.s0[:, self.pos[i]]

    def _bonds(self, i: int) -> np.ndarray:
        nb = neighbours(self.L, i)
        J = self.J
        p = self.pos
        return np.array([J[0, p[i]], J[0, p[nb[1]]], J[1, p[i]], J[1, p[nb[3]]],
                         J[2, p[i]], J[2, p[nb[5]]]], dtype=self.dtype)

    def value(self, i: int, p: int | None = None) -> tuple[np.ndarray, bool]:
        """(spin of site i after the first p steps, tainted)."""
        if p is None:
            p = len(self.steps)
        key = (i, p)
        if key in self.memo:
            return self.memo[key]
        if p == 0:
            out = (self._spin0(i).copy(), False)
        else:
            st = self.steps[p - 1]
            prev, taint = self.value(i, p - 1)
            if st[0] == "renorm":
                s = prev.reshape(3, 1).copy()  # memoised values stay as they were
                O.renormalise(s)
                out = (s.reshape(3), taint)
            else:
                _, sweep, mode, colour, phase = st
                x, y, z = coords(self.L, i)
                if ((x + y + z) & 1) != colour:
                    out = (prev, taint)
                else:
                    nbv = [self.value(j, p - 1) for j in neighbours(self.L, i)]
                    h = O.field(self._bonds(i), np.stack([v for v, _ in nbv]), self.dtype)
                    s, flagged = O.site_update(mode, h, prev, seed=self.seed, sweep=sweep,
                                               site=i, phase=phase, k=self.k, T=self.T,
                                               margin_eps=self.margin_eps, dtype=self.dtype)
                    out = (s, taint or flagged > 0 or any(t for _, t in nbv))
        self.memo[key] = out
        return out
