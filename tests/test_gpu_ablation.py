"""GPU tests of the design-comparison variants (the paper's GM / TEXT / CA / SM / SM4P
designs of §4, Table 2, as sweep flags): each computes the default schedule's spins bit
for bit, and the pass-by-pass variants match the oracle directly."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O
from tests import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hsg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1006_2566_amd as m
    m.lib()
    return m


def variants(m):
    return {"TEXT": m.HSG_SNAKE | m.HSG_STREAM_LOADS, "TEXT-plain": m.HSG_STREAM_LOADS,
            "CA": m.HSG_PLANE_LAUNCH, "CA+S": m.HSG_PLANE_LAUNCH | m.HSG_SNAKE,
            "SM": m.HSG_FUSED | m.HSG_MARCH_PHASE, "SM4P": m.HSG_FUSED,
            "PHASE": m.HSG_SNAKE | m.HSG_PHASE_LAUNCH, "PHASE-plain": m.HSG_PHASE_LAUNCH,
            "PHASE-MC": m.HSG_SNAKE | m.HSG_PHASE_MC, "PHASE-MC-plain": m.HSG_PHASE_MC}


def run(m, L, dtype, flags, *, k, n_or, R, n, hb=False, T=0.4):
    lat = m.Lattice(L, dtype, seed=7)
    lat.sweep(T=T, k=k, n_or=n_or, renorm_every=R, n_sweeps=n, heat_bath=hb, flags=flags)
    return lat.spins.clone(), lat.energy().item()


@pytest.mark.parametrize("L,dtype,k,n_or,R,n,hb", [
    (64, torch.float32, 3, 1, 2, 3, False),
    (64, torch.float64, 0, 2, 1, 3, False),
    (128, torch.float32, 1, 1, 0, 3, True),
    (18, torch.float64, 2, 2, 0, 2, False),
    (256, torch.float32, 4, 1, 10, 2, False),
    (256, torch.float32, 0, 2, 1, 2, False),
    (256, torch.float64, 2, 1, 1, 2, True),
    # renormalisation inside and outside the launches that carry a Monte Carlo pass
    (64, torch.float32, 4, 2, 1, 4, False),
    (128, torch.float64, 2, 1, 3, 4, False),
    (256, torch.float32, 4, 1, 2, 5, False),
    # two over-relaxation phases per sweep at L = 256: the first launched alone, the
    # second carrying the next sweep's colour-0 pass (Metropolis k = 8, heat bath k = 4)
    (256, torch.float32, 8, 2, 3, 3, False),
    (256, torch.float32, 4, 2, 3, 3, True),
])
def test_variants_equal_default_schedule(hsg, L, dtype, k, n_or, R, n, hb):
    ref_s, ref_E = run(hsg, L, dtype, 0, k=k, n_or=n_or, R=R, n=n, hb=hb)
    for name, flags in variants(hsg).items():
        if flags & hsg.HSG_FUSED and not hsg.fused_supported(L):
            continue
        s, E = run(hsg, L, dtype, flags, k=k, n_or=n_or, R=R, n=n, hb=hb)
        assert torch.equal(s, ref_s), name
        if flags & (hsg.HSG_FUSED | hsg.HSG_PHASE_MC):
            assert E == pytest.approx(ref_E, rel=1e-12), name  # summed in another order
        else:
            assert E == ref_E, name


@pytest.mark.parametrize("name", ["TEXT", "CA+S"])
def test_pass_by_pass_variants_match_oracle(hsg, name):
    L, seed = 16, 3
    spins, J = inputs.random_state(L, 41, np.float32)
    lat = hsg.Lattice(L, torch.float32, seed=seed, init=None)
    lat.load(torch.from_numpy(spins), torch.from_numpy(J))
    lat.sweep(T=0.5, k=3, n_or=1, renorm_every=0, n_sweeps=2, flags=variants(hsg)[name])
    got = lat.export()[0].cpu().numpy()
    s = spins.copy()
    taint = np.zeros(L ** 3, dtype=np.uint8)
    O.sweep(L, seed, s, J, T=0.5, k=3, n_or=1, n_sweeps=2, E=O.energy(L, spins, J), taint=taint)
    ok = taint == 0
    assert ok.sum() >= 0.99 * L ** 3
    assert np.abs(got[:, ok] - s[:, ok]).max() <= 1e-5


@pytest.mark.parametrize("dtype,hb,R,n", [(np.float32, False, 1, 2), (np.float64, False, 1, 2),
                                          (np.float64, True, 2, 3), (np.float64, True, 0, 3)])
def test_phase_with_monte_carlo_pass_matches_oracle(hsg, dtype, hb, R, n):
    """HSG_PHASE_MC straight against the oracle at L = 64: every sweep but the last ends
    with a launch that also runs the next sweep's colour-0 pass (and the renormalisation
    due between them).  Metropolis runs two sweeps, so that the sites tainted by
    decisions within 1e-6 of their threshold stay below 1%; heat bath makes no such
    decisions and runs three, in binary64 (binary32 heat-bath draws go through library
    logarithms that may differ from the host's by an ulp, which later sweeps amplify; the
    binary32 draws are checked pass by pass against the oracle elsewhere, and the launch
    against the pass-by-pass schedule bit for bit above)."""
    L, seed = 64, 5
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    spins, J = inputs.random_state(L, 43, dtype)
    lat = hsg.Lattice(L, tdt, seed=seed, init=None)
    lat.load(torch.from_numpy(spins), torch.from_numpy(J))
    E0 = lat.energy().item()
    lat.sweep(T=0.5, k=3, n_or=1, renorm_every=R, n_sweeps=n, heat_bath=hb,
              flags=hsg.HSG_SNAKE | hsg.HSG_PHASE_MC)
    got = lat.export()[0].cpu().numpy()
    s = spins.copy()
    taint = np.zeros(L ** 3, dtype=np.uint8)
    r = O.sweep(L, seed, s, J, T=0.5, k=3, n_or=1, renorm_every=R, n_sweeps=n, E=E0,
                heat_bath=hb, taint=taint)
    ok = taint == 0
    assert ok.sum() >= 0.99 * L ** 3
    tol = 1e-5 if dtype == np.float32 else 1e-12
    assert np.abs(got[:, ok] - s[:, ok]).max() <= tol
    if r["n_flagged"] == 0:
        assert abs(lat.energy().item() - r["E"]) <= tol * abs(r["E"])


def test_phase_with_monte_carlo_pass_large_lattice(hsg):
    """HSG_PHASE_MC at L = 512 (4096 workgroups per launch) against the pass-by-pass
    schedule: six sweeps, renormalisation due after sweeps 1 and 3 (inside launches) and
    after sweep 5, the call's last."""
    L = 512
    ref_s, ref_E = run(hsg, L, torch.float32, hsg.HSG_SNAKE, k=2, n_or=1, R=2, n=6)
    s, E = run(hsg, L, torch.float32, hsg.HSG_SNAKE | hsg.HSG_PHASE_MC, k=2, n_or=1, R=2, n=6)
    assert torch.equal(s, ref_s)
    assert E == pytest.approx(ref_E, rel=1e-12)
    del ref_s, s
    torch.cuda.empty_cache()
