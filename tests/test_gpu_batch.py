"""GPU tests of the batched form: every chain of a batch computes what the single-lattice
path and the oracle compute for that lattice; parallel tempering follows the oracle's
exchange step; graph replays equal eager runs; results do not depend on the
workgroup size."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F32, F64 = np.float32, np.float64


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1006_2566_amd as hsg
    from paper_1006_2566_amd import batch as B
    hsg.lib()
    return hsg, B


def mixed_specs(B, k=3, n_or=1, heat_last=True):
    Ls = [4, 8, 8, 12, 16, 24, 32, 6, 10, 48]
    specs = []
    for i, L in enumerate(Ls):
        group = 100 + (i if i not in (2,) else 1)  # chains 1 and 2 share couplings
        specs.append(B.ChainSpec(L=L, seed=1000 + 17 * i, J_group=group, J_seed=77 + i,
                                 T=0.3 + 0.1 * i, k=k, n_or=n_or, renorm_every=2,
                                 heat_bath=(heat_last and i == len(Ls) - 1)))
    return specs


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_batch_chain_equals_single_lattice(mods, dtype):
    hsg, B = mods
    specs = mixed_specs(B)
    b = B.Batch(specs, dtype=dtype, threads=256)
    init = [b.export_chain(c) for c in range(b.n)]
    E0 = b.energies().cpu().numpy()
    b.sweep(3)
    E_b = b.energies().cpu().numpy()
    sw = b.sweep_ctr.cpu().numpy()
    assert (sw == 3).all()
    for c, sp in enumerate(specs):
        lat = hsg.Lattice(sp.L, dtype, seed=sp.seed, init=None)
        lat.load(init[c][0], init[c][1])
        assert abs(lat.energy().item() - E0[c]) <= 1e-12 * max(1, abs(E0[c]))
        lat.sweep(T=sp.T, k=sp.k, n_or=sp.n_or, renorm_every=sp.renorm_every, n_sweeps=3,
                  heat_bath=sp.heat_bath)
        s_single = lat.export()[0]
        s_batch = b.export_chain(c)[0]
        assert torch.equal(s_single, s_batch), f"chain {c} L={sp.L}"
        assert abs(lat.energy().item() - E_b[c]) <= 1e-12 * max(1, abs(E_b[c]))
    # shared couplings really are shared
    assert torch.equal(b.export_chain(1)[1], b.export_chain(2)[1])


def test_batch_init_matches_oracle(mods):
    """Philox initial state of every chain (spins from its seed, couplings from the
    seed of its group's first chain) against the oracle's."""
    hsg, B = mods
    specs = mixed_specs(B, k=2, n_or=1, heat_last=False)
    b = B.Batch(specs, dtype=torch.float32)
    group_seed = {}
    for sp in specs:
        group_seed.setdefault(sp.J_group, sp.J_seed)
    for c, sp in enumerate(specs):
        s0, _ = O.init(sp.L, sp.seed, F32)
        _, J = O.init(sp.L, group_seed[sp.J_group], F32)
        gs, gJ = (t.cpu().numpy() for t in b.export_chain(c))
        np.testing.assert_array_equal(gs, s0)
        # couplings go through log() in Box-Muller: an ulp apart at most
        np.testing.assert_allclose(gJ, J, rtol=4e-7, atol=4e-7)


@pytest.mark.parametrize("dtype", [F32, F64])
def test_batch_sweep_matches_oracle(mods, dtype):
    """Every chain, loaded from seeded inputs, against the oracle after 3 sweeps."""
    from tests import inputs
    hsg, B = mods
    specs = mixed_specs(B, k=2, n_or=1, heat_last=False)
    b = B.Batch(specs, dtype=torch.float32 if dtype == F32 else torch.float64)
    states = {}
    for c, sp in enumerate(specs):
        s, J = inputs.random_state(sp.L, 40 + c, dtype)
        if sp.J_group in states:  # shared couplings: reuse the group's
            J = states[sp.J_group]
        states.setdefault(sp.J_group, J)
        b.load_chain(c, torch.from_numpy(s), torch.from_numpy(J))
        states[c] = (s, J)
    b.sweep(3)
    E = b.energies().cpu().numpy()
    tol = 1e-5 if dtype == F32 else 1e-12
    for c, sp in enumerate(specs):
        s0, J = states[c]
        s = s0.copy()
        taint = np.zeros(sp.L ** 3, dtype=np.uint8)
        r = O.sweep(sp.L, sp.seed, s, J, T=sp.T, k=sp.k, n_or=sp.n_or,
                    renorm_every=sp.renorm_every, n_sweeps=3, E=O.energy(sp.L, s0, J),
                    taint=taint)
        got = b.export_chain(c)[0].cpu().numpy()
        ok = taint == 0
        err = float(np.abs(got[:, ok] - s[:, ok]).max()) if ok.any() else 0.0
        print(f"[parity] batch chain {c} L={sp.L}: max|d|={err:.2e} tainted={int((~ok).sum())}")
        assert err <= tol and (~ok).sum() <= max(8, 0.05 * sp.L ** 3)
        if not taint.any():
            assert abs(E[c] - r["E"]) <= tol * abs(r["E"])


@pytest.mark.parametrize("threads", [64, 512, 1024])
def test_batch_independent_of_workgroup_size(mods, threads):
    hsg, B = mods
    specs = mixed_specs(B)
    ref = B.Batch(specs, threads=256)
    other = B.Batch(specs, threads=threads)
    ref.sweep(4)
    other.sweep(4)
    assert torch.equal(ref.spins, other.spins)
    assert torch.allclose(ref.E, other.E, rtol=1e-12, atol=0)


def test_batch_remaining_budget(mods):
    hsg, B = mods
    specs = mixed_specs(B)[:4]
    b = B.Batch(specs, track_remaining=True)
    b.remaining.copy_(torch.tensor([0, 1, 5, 3], dtype=torch.int32))
    b.sweep(4)
    assert b.sweep_ctr.cpu().tolist() == [0, 1, 4, 3]
    assert b.remaining.cpu().tolist() == [0, 0, 1, 0]
    b.sweep(4)
    assert b.sweep_ctr.cpu().tolist() == [0, 1, 5, 3]


def _seeded_states(B, b, specs):
    """Load every chain from seeded inputs (couplings shared within a group); returns
    the host copies."""
    from tests import inputs
    states, group_J = {}, {}
    for c, sp in enumerate(specs):
        s, J = inputs.random_state(sp.L, 500 + c, F32)
        J = group_J.setdefault(sp.J_group, J)
        b.load_chain(c, torch.from_numpy(s), torch.from_numpy(J))
        states[c] = [s.copy(), J, O.energy(sp.L, s, J)]
    return states


def _oracle_pt(specs, states, ladders, betas, seed, n_cycles, spe):
    """Oracle run of the same schedule: every chain sweeps at its slot's temperature,
    then each ladder takes one exchange round with the tracked energies."""
    chain_at_slot = ladders.copy()
    for cycle in range(n_cycles):
        beta_of_chain = np.zeros(len(specs))
        for l in range(ladders.shape[0]):
            for t in range(ladders.shape[1]):
                beta_of_chain[chain_at_slot[l, t]] = betas[t]
        for c, sp in enumerate(specs):
            s, J, E = states[c]
            r = O.sweep(sp.L, sp.seed, s, J, T=1.0 / beta_of_chain[c], k=sp.k, n_or=sp.n_or,
                        n_sweeps=spe, sweep0=cycle * spe, E=E)
            states[c][2] = r["E"]
        Es = np.array([states[c][2] for c in range(len(specs))])
        for l in range(ladders.shape[0]):
            row = np.ascontiguousarray(chain_at_slot[l])
            O.pt_swap(betas, Es, row, seed=seed, stream_id=l, round_=cycle)
            chain_at_slot[l] = row
    return states, chain_at_slot


def test_parallel_tempering_matches_oracle(mods):
    hsg, B = mods
    specs, ladders, betas, pairs = B.pt_workload(n_samples=3, Ls=(4, 6), replicas=2, n_temps=5,
                                                 T_min=0.3, T_max=2.0, k=2, base_seed=5)
    b = B.Batch(specs)
    states = _seeded_states(B, b, specs)
    pt = B.Tempering(b, ladders, betas, seed=99)
    n_cycles, spe = 4, 2
    for _ in range(n_cycles):
        b.sweep(spe)
        pt.exchange()
    states, cas = _oracle_pt(specs, states, ladders, betas, 99, n_cycles, spe)
    np.testing.assert_array_equal(pt.chain_at_slot.cpu().numpy(), cas)
    E = b.E.cpu().numpy()
    for c, sp in enumerate(specs):
        got = b.export_chain(c)[0].cpu().numpy()
        assert np.abs(got - states[c][0]).max() <= 1e-5, c
        assert abs(E[c] - states[c][2]) <= 1e-5 * abs(states[c][2])
    # overlap between the two replicas, slot by slot
    q = pt.overlap(pairs).cpu().numpy()
    for p, (la, lb) in enumerate(pairs):
        for t in range(ladders.shape[1]):
            a, c2 = cas[la, t], cas[lb, t]
            Q, ma, mb = O.overlap(specs[a].L, b.export_chain(a)[0].cpu().numpy(),
                                  b.export_chain(c2)[0].cpu().numpy())
            np.testing.assert_allclose(q[p, t, :9], Q.ravel(), atol=1e-13)
            np.testing.assert_allclose(q[p, t, 9:12], ma, atol=1e-13)


def test_graph_replay_equals_eager(mods):
    hsg, B = mods
    specs, ladders, betas, pairs = B.pt_workload(n_samples=4, Ls=(8, 12), replicas=2, n_temps=4,
                                                 T_min=0.2, T_max=1.0, k=2, base_seed=9)
    ba = B.Batch(specs)
    bb = B.Batch(specs)
    ra = B.PTRunner(ba, B.Tempering(ba, ladders, betas, seed=3), pairs, 3, 2, use_graph=True)
    rb = B.PTRunner(bb, B.Tempering(bb, ladders, betas, seed=3), pairs, 3, 2, use_graph=False)
    for cycle in range(4):
        ra.run_cycle()
        rb.run_cycle()
        torch.cuda.synchronize()
        # eager work in between replays
        _ = (ba.E * 2).sum().item()
        assert torch.equal(ba.spins, bb.spins), cycle
        assert torch.equal(ba.E, bb.E), cycle
        assert torch.equal(ra.pt.chain_at_slot, rb.pt.chain_at_slot), cycle
        assert torch.equal(ra.q, rb.q), cycle
    assert int(ra.pt.round.item()) == 4 * 2


def test_autotune_batch_threads_restores_state(mods, tmp_path):
    """Tuning times real sweeps of the batch, then puts every chain back as it was."""
    hsg, B = mods
    from paper_1006_2566_amd import autotune as A
    b = B.Batch(mixed_specs(B), track_remaining=True)
    b.remaining.fill_(9)
    before = (b.spins.clone(), b.E.clone(), b.sweep_ctr.clone(), b.remaining.clone())
    t = A.batch_threads(b, path=str(tmp_path / "tune.json"))
    assert t in (64, 128, 256, 512, 1024) and b.threads == t
    assert torch.equal(b.spins, before[0]) and torch.equal(b.E, before[1])
    assert torch.equal(b.sweep_ctr, before[2]) and torch.equal(b.remaining, before[3])
    assert A.load_cache(str(tmp_path / "tune.json"))[A.device_key()]


def test_autotune_sweep_flags(mods, tmp_path):
    hsg, B = mods
    from paper_1006_2566_amd import autotune as A
    phase = hsg.HSG_SNAKE | hsg.HSG_PHASE_LAUNCH
    f = A.sweep_flags(64, k=2, n_or=1, path=str(tmp_path / "tune.json"))
    assert f in (0, hsg.HSG_SNAKE, phase, hsg.HSG_SNAKE | hsg.HSG_PHASE_MC)
    f = A.sweep_flags(256, k=1, n_or=1, path=str(tmp_path / "tune.json"))
    assert f in (0, hsg.HSG_SNAKE, phase, hsg.HSG_SNAKE | hsg.HSG_PHASE_MC, hsg.HSG_FUSED)
    f = A.sweep_flags(96, k=1, n_or=0, path=str(tmp_path / "tune.json"))
    assert f in (0, hsg.HSG_SNAKE)
