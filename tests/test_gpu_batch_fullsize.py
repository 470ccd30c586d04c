"""The batched workload at its full size, on sampled ladders.

The whole parallel-tempering workload the bench times (256 disorder samples, L drawn from
{16, 24, 32, 48}, 2 replicas x 24 geometric temperatures in [0.12, 0.5], binary32,
Metropolis k = 4: 12288 chains, 5.3e8 spins) is initialised on the GPU and advanced by the
batched sweep launch and the exchange kernel, three blocks of two sweeps each followed by
an exchange round (the bench runs blocks of ten: the same launches with a longer count;
shorter blocks keep the taint cones of flagged decisions small at T = 0.12).  Three
ladders (the first of a sample with L = 16, 32 and 48) are then recomputed by the oracle
from the GPU's initial state of their chains -- each chain swept at its slot's
temperature, then the ladder's exchange round with the tracked energies -- and compared:
the chain in every slot, every spin within 1e-5 outside the oracle's taint cones
(decisions within 1e-6 of their threshold, counted), and the tracked energy of every
chain without flagged decisions."""
from __future__ import annotations

import numpy as np
import pytest

import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1006_2566_amd as hsg
    from paper_1006_2566_amd import batch as B
    hsg.lib()
    return hsg, B


def test_full_batched_workload_on_sampled_ladders(mods):
    hsg, B = mods
    specs, ladders, betas, pairs = B.pt_workload()
    assert len(specs) == 12288
    torch.cuda.empty_cache()
    b = B.Batch(specs)
    pt = B.Tempering(b, ladders, betas, seed=1)
    # the first ladder of a sample of each of three sizes
    picks = []
    for L in (16, 32, 48):
        picks.append(next(l for l in range(ladders.shape[0]) if specs[ladders[l, 0]].L == L))
    chains = sorted({int(c) for l in picks for c in ladders[l]})
    start = {c: [t.cpu().numpy().copy() for t in b.export_chain(c)] for c in chains}
    n_cycles, spe = 3, 2
    for _ in range(n_cycles):
        b.sweep(spe)
        pt.exchange()
    torch.cuda.synchronize()
    cas_gpu = pt.chain_at_slot.cpu().numpy()
    E_gpu = b.E.cpu().numpy()
    got = {c: b.export_chain(c)[0].cpu().numpy() for c in chains}
    print(f"ladders {picks}: {len(chains)} chains", flush=True)

    # oracle: the same schedule for the sampled ladders
    states = {}
    for c in chains:
        s, J = start[c]
        s, J = np.ascontiguousarray(s), np.ascontiguousarray(J)
        states[c] = [s, J, O.energy(specs[c].L, s, J), np.zeros(specs[c].L ** 3, np.uint8)]
    cas = ladders.copy()
    flagged = 0
    for cycle in range(n_cycles):
        for l in picks:
            for t, c in enumerate(cas[l]):
                sp = specs[c]
                s, J, E, taint = states[c]
                r = O.sweep(sp.L, sp.seed, s, J, T=1.0 / betas[t], k=sp.k, n_or=sp.n_or,
                            n_sweeps=spe, sweep0=cycle * spe, E=E, taint=taint)
                states[c][2] = r["E"]
                flagged += r["n_flagged"]
        Es = np.zeros(len(specs))
        for c in chains:
            Es[c] = states[c][2]
        for l in picks:
            row = np.ascontiguousarray(cas[l])
            O.pt_swap(betas, Es, row, seed=1, stream_id=l, round_=cycle)
            cas[l] = row
    print(f"flagged decisions: {flagged}")
    for l in picks:
        np.testing.assert_array_equal(cas_gpu[l], cas[l], err_msg=f"ladder {l}")
    compared = total = 0
    for c in chains:
        s, J, E, taint = states[c]
        ok = taint == 0
        compared += int(ok.sum())
        total += ok.size
        np.testing.assert_allclose(got[c][:, ok], s[:, ok], rtol=0, atol=1e-5, err_msg=f"chain {c}")
        if not taint.any():
            assert abs(E_gpu[c] - E) <= 1e-9 * abs(E), (c, E_gpu[c], E)
    print(f"{compared} of {total} sites compared (the rest in taint cones)")
    assert compared >= 0.9 * total
    del b, pt
    torch.cuda.empty_cache()
