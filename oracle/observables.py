"""Spin-glass observables from the tensor overlap, written out in numpy (binary64).

TEST INFRASTRUCTURE ONLY: the definitions the GPU library's Fourier-overlap entry
points and the package's estimators must reproduce.  Only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use it.

The paper (Bernaschi, Parisi & Parisi, arXiv:1006.2566) simulates the model of §2 but
defines no observable; the ones here are the standard finite-size analysis of vector
spin glasses built on the overlap of two real replicas a, b with the same couplings:

* local overlap tensor  q_r^{mu nu} = a_r^mu b_r^nu  (3 x 3 per site r = (x, y, z));
* its Fourier components  Q^{mu nu}(k) = (1/N) sum_r q_r^{mu nu} exp(+i k.r)  at k = 0
  and at the three smallest non-zero wave-vectors k_d = (2 pi / L) e_d;
* q2(k) = sum_{mu nu} |Q^{mu nu}(k)|^2, with q2(k_min) averaged over d = x, y, z;
* chi_SG(k) = N <q2(k)>;
* second-moment correlation length  xi = sqrt(chi(0) / chi(k_min) - 1) / (2 sin(k_min / 2));
* Binder cumulant of the 9-component (n = 3) tensor order parameter
  g = (n^2 + 2)/2 - (n^2/2) <q2(0)^2> / <q2(0)>^2 = (11 - 9 <q2^2>/<q2>^2) / 2,
  which is 1 for a frozen overlap and 0 for 9 independent Gaussian components.

Record layout (65 values, as the library writes them):
  [0, 9)               Q^{mu nu}(0), row-major (mu = row)
  [9 + 18d, 18 + 18d)  Re Q^{mu nu}(k_d),  d = 0, 1, 2 for x, y, z
  [18 + 18d, 27 + 18d) Im Q^{mu nu}(k_d)
  [63]                 q2(0)
  [64]                 q2(k_min) = (1/3) sum_d q2(k_d)

Arrays use the canonical layout of the oracle: (3, N) with site i = x + L*y + L*L*z.
"""
from __future__ import annotations

import numpy as np

N_VALUES = 65


def overlap_fourier(L: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """The 65-value record of two configurations a, b (shape (3, L^3))."""
    N = L ** 3
    # canonical i = x + L*y + L*L*z, so a reshape to (L, L, L) indexes [z, y, x]
    A = np.asarray(a, dtype=np.float64).reshape(3, L, L, L)
    B = np.asarray(b, dtype=np.float64).reshape(3, L, L, L)
    wave = np.exp(2j * np.pi * np.arange(L) / L)  # exp(i k_min r_d), r_d = 0 .. L-1
    out = np.zeros(N_VALUES)
    for mu in range(3):
        for nu in range(3):
            q = A[mu] * B[nu]                       # q_r^{mu nu}, [z, y, x]
            m = 3 * mu + nu
            out[m] = q.sum() / N
            # d = 0 (x) sums against axis 2, d = 1 (y) axis 1, d = 2 (z) axis 0
            for d, axis in ((0, 2), (1, 1), (2, 0)):
                shape = [1, 1, 1]
                shape[axis] = L
                Qk = (q * wave.reshape(shape)).sum() / N
                out[9 + 18 * d + m] = Qk.real
                out[18 + 18 * d + m] = Qk.imag
    out[63] = np.sum(out[0:9] ** 2)
    out[64] = np.sum(out[9:63] ** 2) / 3.0
    return out


def chi_sg(records: np.ndarray, N: int) -> tuple[float, float]:
    """(chi_SG(0), chi_SG(k_min)) from a series of records (shape (n, 65))."""
    r = np.asarray(records, dtype=np.float64).reshape(-1, N_VALUES)
    return N * float(np.mean(r[:, 63])), N * float(np.mean(r[:, 64]))


def xi_second_moment(chi0: float, chik: float, L: int) -> float:
    """Second-moment correlation length; NaN when chi(0) < chi(k_min)."""
    ratio = chi0 / chik - 1.0
    if not ratio >= 0.0:
        return float("nan")
    return float(np.sqrt(ratio) / (2.0 * np.sin(np.pi / L)))


def binder_g(records: np.ndarray) -> float:
    """Binder cumulant of the tensor overlap from a series of records."""
    q2 = np.asarray(records, dtype=np.float64).reshape(-1, N_VALUES)[:, 63]
    return float(0.5 * (11.0 - 9.0 * np.mean(q2 ** 2) / np.mean(q2) ** 2))
