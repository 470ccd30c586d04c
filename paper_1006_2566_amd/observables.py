"""Spin-glass estimators over a series of Fourier-overlap records.

The GPU writes one 65-value record per replica pair and measurement
(hsg_overlap_fourier / hsg_batch_overlap_fourier / hsg_pt_overlap_fourier): Q(0),
Re/Im Q(k_d) for d = x, y, z, q2(0) = sum |Q(0)|^2 and q2(k_min) = (1/3) sum_d sum
|Q(k_d)|^2.  This module keeps running moments of q2 over measurements (a few numbers
per pair and temperature, on the host) and turns them into the standard estimators
of vector spin glasses:

* chi_SG(k) = N [<q2(k)>]                        (k = 0 and k_min = 2 pi / L)
* xi = sqrt(chi(0) / chi(k_min) - 1) / (2 sin(pi / L))   (second-moment length)
* g = (11 - 9 [<q2(0)^2>] / [<q2(0)>]^2) / 2             (Binder cumulant, n = 3)

where <.> is the thermal average of one pair and [.] the average over pairs
(disorder samples) of one lattice size.  The paper's model (§2) is what these
measure; the paper itself defines no observable.
"""
from __future__ import annotations

import math

import numpy as np

Q2_0, Q2_KMIN = 63, 64


class OverlapMoments:
    """Running sums of q2(0), q2(0)^2 and q2(k_min) per record slot (for example
    [pair, temperature])."""

    def __init__(self, shape):
        self.shape = tuple(shape)
        self.n = 0
        self.s_q2 = np.zeros(self.shape)
        self.s_q4 = np.zeros(self.shape)
        self.s_q2k = np.zeros(self.shape)

    def add(self, records) -> None:
        """Adds one measurement: records of shape shape + (65,) (tensor or array)."""
        r = records.detach().cpu().numpy() if hasattr(records, "detach") else np.asarray(records)
        r = r.reshape(self.shape + (65,))
        q2 = r[..., Q2_0]
        self.s_q2 += q2
        self.s_q4 += q2 * q2
        self.s_q2k += r[..., Q2_KMIN]
        self.n += 1

    def thermal(self):
        """Per-slot thermal averages (<q2(0)>, <q2(0)^2>, <q2(k_min)>)."""
        if self.n == 0:
            raise ValueError("no measurement added")
        return self.s_q2 / self.n, self.s_q4 / self.n, self.s_q2k / self.n


def estimators(q2: np.ndarray, q4: np.ndarray, q2k: np.ndarray, L: int) -> dict:
    """chi(0), chi(k_min), xi and g from thermal averages of the pairs of one lattice
    size (arrays over pairs, averaged here over their first axis)."""
    N = L ** 3
    m2, m4, m2k = (np.mean(np.asarray(v, dtype=np.float64), axis=0) for v in (q2, q4, q2k))
    chi0, chik = N * m2, N * m2k
    ratio = chi0 / chik - 1.0
    with np.errstate(invalid="ignore"):
        xi = np.where(ratio >= 0.0, np.sqrt(np.maximum(ratio, 0.0)), np.nan) / (
            2.0 * math.sin(math.pi / L))
    g = 0.5 * (11.0 - 9.0 * m4 / (m2 * m2))
    return {"chi0": chi0, "chik": chik, "xi": xi, "g": g}


def by_size(moments: OverlapMoments, L_of_pair) -> dict:
    """Disorder averages per lattice size: {L: estimators over the pairs of that L}.
    The first axis of the moments' slots is the pair; any further axes (temperature)
    are kept."""
    q2, q4, q2k = moments.thermal()
    Ls = np.asarray(L_of_pair)
    return {int(L): estimators(q2[Ls == L], q4[Ls == L], q2k[Ls == L], int(L))
            for L in np.unique(Ls)}
