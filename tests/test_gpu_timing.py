"""The measurement form hsg_sweep_timed: it computes exactly what hsg_sweep computes,
reports the call's launches in order with their kinds, and gives each a positive
event-timed duration.  The benchmark takes its per-kernel durations from it."""
from __future__ import annotations

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hsg():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1006_2566_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("L,k,n_or,n,flags_name,expected", [
    # the benchmark traversal: colour-0 pass, then per sweep the colour-1 pass and the
    # phase launch carrying the next colour-0 pass; three phase launches would leave the
    # spins in the second array, so the last phase runs as two passes; then the fold
    (256, 4, 1, 3, "mc", [1, 1, 4, 1, 4, 1, 2, 2, 0]),
    (256, 4, 1, 2, "mc", [1, 1, 4, 1, 3, 0]),
    (64, 1, 1, 2, "phase", [1, 1, 3, 1, 1, 3, 0]),
    (32, 2, 1, 1, "plain", [1, 1, 2, 2, 0]),
])
def test_sweep_timed_equals_sweep(hsg, L, k, n_or, n, flags_name, expected):
    flags = {"mc": hsg.HSG_SNAKE | hsg.HSG_PHASE_MC,
             "phase": hsg.HSG_SNAKE | hsg.HSG_PHASE_LAUNCH, "plain": hsg.HSG_SNAKE}[flags_name]
    a = hsg.Lattice(L, torch.float32, seed=3)
    b = hsg.Lattice(L, torch.float32, seed=3)
    a.sweep(T=0.5, k=k, n_or=n_or, n_sweeps=n, flags=flags)
    rec = b.sweep_timed(T=0.5, k=k, n_or=n_or, n_sweeps=n, flags=flags)
    print(f"[timed] L={L} k={k} n_or={n_or} n={n} {flags_name}: "
          + " ".join(f"{hsg.LAUNCH_NAMES[kd]}:{ms * 1e3:.1f}us" for kd, ms in rec), flush=True)
    assert torch.equal(a.spins, b.spins)
    assert a.sweep_index == b.sweep_index == n
    assert abs(a.energy().item() - b.energy().item()) <= 1e-12 * abs(a.energy().item())
    assert [kd for kd, _ in rec] == expected
    assert all(ms > 0 for _, ms in rec)


def test_sweep_timed_capacity_limits_the_record(hsg):
    lat = hsg.Lattice(16, torch.float32, seed=4)
    rec = lat.sweep_timed(T=1.0, k=1, n_sweeps=5, capacity=3)
    assert len(rec) == 3 and lat.sweep_index == 5
    lat.sweep_timed(T=1.0, k=1, n_sweeps=1, capacity=0)
    assert lat.sweep_index == 6
