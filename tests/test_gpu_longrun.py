"""Long-run agreement of the equilibrium energy: the GPU's Markov chain and the oracle's,
started from the same state on the same couplings but driven by independent Philox
streams (different seeds), must give the same mean energy per site within 3 combined
standard errors.  This pins the physics of the sweep (the Hamiltonian of §2 eq. 1,
the local field of eq. 2, Metropolis with k hits and the over-relaxation of §4) beyond
one sweep: a wrong acceptance rule, a missed term of the field or a mis-scaled
temperature would move the equilibrium energy by many standard errors.

Errors come from a binning analysis: the series of per-sweep energies is cut into
2^b bins for growing bin lengths, and the standard error of the mean is taken at the
largest bin length that still leaves 32 bins (the plateau for correlation times well
below that length).
"""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

BURN_IN = 2000
MEASURE = 1 << 14


def binned_mean_se(x: np.ndarray) -> tuple[float, float, int]:
    """(mean, standard error, bin length) of a correlated series by binning."""
    x = np.asarray(x, dtype=np.float64)
    mean = float(x.mean())
    best, blen = 0.0, 1
    b = 1
    while x.size // b >= 32:
        nb = x.size // b
        means = x[:nb * b].reshape(nb, b).mean(axis=1)
        se = float(means.std(ddof=1) / np.sqrt(nb))
        if se > best:
            best, blen = se, b
        b *= 2
    return mean, best, blen


def oracle_series(L, seed, spins, J, *, T, k, n_or):
    s = spins.copy()
    E = O.energy(L, s, J)
    out = np.empty(MEASURE)
    for n in range(BURN_IN + MEASURE):
        E = O.sweep(L, seed, s, J, T=T, k=k, n_or=n_or, n_sweeps=1, sweep0=n, E=E)["E"]
        if n >= BURN_IN:
            out[n - BURN_IN] = E
    return out / L ** 3


def gpu_series(hsg, L, seed, spins, J, *, T, k, n_or):
    lat = hsg.Lattice(L, torch.float32, seed=seed, init=None)
    lat.load(torch.from_numpy(spins), torch.from_numpy(J))
    lib = hsg.lib()
    flags = hsg.default_flags(L, torch.float32)
    p = hsg._SweepParams(float(T), int(k), int(n_or), 0, flags)
    Es = torch.empty(MEASURE, dtype=torch.float64, device="cuda")
    st = hsg._stream(None)
    base = Es.data_ptr()
    for n in range(BURN_IN + MEASURE):
        hsg.check(lib.hsg_sweep(ctypes.byref(lat._d), ctypes.byref(p), 1, st))
        if n >= BURN_IN:
            hsg.check(lib.hsg_energy(ctypes.byref(lat._d), 0,
                                     ctypes.c_void_p(base + 8 * (n - BURN_IN)), st))
    out = Es.cpu().numpy()
    E_rec = lat.energy(recompute=True).item()
    assert abs(out[-1] - E_rec) <= 1e-5 * abs(E_rec)  # tracked = recomputed at the end
    return out / L ** 3


@pytest.fixture(scope="module")
def hsg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1006_2566_amd as m
    m.lib()
    return m


CASES = [  # L, T, k, n_or
    (8, 0.5, 1, 0), (8, 1.0, 1, 0), (8, 0.5, 4, 1), (8, 1.0, 4, 1),
    (16, 0.5, 1, 0), (16, 1.0, 1, 0), (16, 0.5, 4, 1), (16, 1.0, 4, 1),
]


@pytest.mark.parametrize("L,T,k,n_or", CASES)
def test_mean_energy_agrees_with_oracle(hsg, L, T, k, n_or):
    spins, J = O.init(L, 100 + L, np.float32)  # one disorder sample, one start
    seed_gpu, seed_cpu = 7000 + 10 * L + k, 9000 + 10 * L + k
    e_gpu = gpu_series(hsg, L, seed_gpu, spins, J, T=T, k=k, n_or=n_or)
    e_cpu = oracle_series(L, seed_cpu, spins, J, T=T, k=k, n_or=n_or)
    mg, sg, bg = binned_mean_se(e_gpu)
    mc, sc, bc = binned_mean_se(e_cpu)
    z = (mg - mc) / np.hypot(sg, sc)
    print(f"[longrun] L={L} T={T} k={k} n_or={n_or}: <e> gpu {mg:.6f} +- {sg:.1e} (bin {bg}) "
          f"oracle {mc:.6f} +- {sc:.1e} (bin {bc}) z={z:+.2f}", flush=True)
    assert abs(z) < 3.0
    # the error bars resolve the physics: well below the gap to the infinite-temperature
    # energy (0) and to the ground-state scale (about -1 per site)
    assert max(sg, sc) < 0.01 * abs(mc)
