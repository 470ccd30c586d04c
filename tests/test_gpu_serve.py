"""GPU tests of the served form: results do not depend on what else is resident
(alone vs in the mix), match the single-lattice path (also on the served stream's own mix
of sizes and arrivals), admission by footprint waits instead of failing, and the
multi-lattice pass sweep equals the chain-per-workgroup sweep."""
from __future__ import annotations

import math

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
    from paper_1006_2566_amd import serve as S
    hsg.lib()
    return hsg, B, S


def small_trace(S, n=14, seed=4):
    rng = np.random.default_rng(seed)
    Ls = [8, 16, 32, 64]
    return [S.Request(rid=r, seed=5000 + r, L=int(rng.choice(Ls)), T=float(rng.uniform(0.1, 1.0)),
                      sweeps=int(rng.integers(5, 60)), k=int(rng.choice([1, 4])),
                      arrival=0.001 * r) for r in range(n)]


def test_results_same_alone_and_in_mix(mods):
    hsg, B, S = mods
    trace = small_trace(S)
    mix = {r.rid: r for r in S.Server(hbm_budget=256 << 20, n_slots=64, step_sweeps=7).run(
        trace, realtime=False)}
    assert sorted(mix) == [r.rid for r in trace]
    for req in trace[:6]:
        alone = S.Server(hbm_budget=64 << 20, n_slots=4, step_sweeps=5).run([req],
                                                                          realtime=False)[0]
        a, b = alone, mix[req.rid]
        print(f"[serve] rid={req.rid} L={req.L} E alone={a.E:.9f} mix={b.E:.9f}")
        # spins identical; E sums binary64 atomics in a different order
        np.testing.assert_array_equal(a.m, b.m)
        assert abs(a.E - b.E) <= 1e-12 * max(1.0, abs(a.E))


def test_results_match_single_lattice_path(mods):
    hsg, B, S = mods
    trace = small_trace(S, n=6, seed=11)
    res = {r.rid: r for r in S.Server(hbm_budget=256 << 20, n_slots=16, step_sweeps=9).run(
        trace, realtime=False)}
    for req in trace:
        lat = hsg.Lattice(req.L, torch.float32, seed=req.seed)
        lat.sweep(T=req.T, k=req.k, n_sweeps=req.sweeps)
        s = lat.export()[0].double()
        m = (s.mean(dim=1)).cpu().numpy()
        E = lat.energy().item()
        np.testing.assert_allclose(res[req.rid].m, m, rtol=0, atol=1e-12)
        assert abs(res[req.rid].E - E) <= 1e-10 * max(1.0, abs(E))


def test_served_stream_matches_single_lattice_path(mods):
    """The served stream's own mix (L in {8, ..., 96}, k in {1, 4}, Poisson arrivals at
    200 per second, served in real time so requests join while others run), with the
    sweep counts capped at 300: every result equals the single-lattice path's."""
    hsg, B, S = mods
    trace = S.poisson_trace(n=60, rate=200.0, seed=1)
    for r in trace:
        r.sweeps = min(r.sweeps, 300)
    assert {r.L for r in trace} == {8, 16, 32, 64, 96}
    srv = S.Server(hbm_budget=1 << 30, n_slots=64, step_sweeps=16, tile_sites=512)
    res = {r.rid: r for r in srv.run(trace, realtime=True)}
    assert sorted(res) == [r.rid for r in trace]
    assert all(r.status == "ok" and r.sweeps_done == q.sweeps for q in trace
               for r in [res[q.rid]])
    for req in trace:
        lat = hsg.Lattice(req.L, torch.float32, seed=req.seed)
        lat.sweep(T=req.T, k=req.k, n_sweeps=req.sweeps)
        m = lat.export()[0].double().mean(dim=1).cpu().numpy()
        E = lat.energy().item()
        np.testing.assert_allclose(res[req.rid].m, m, rtol=0, atol=1e-12, err_msg=str(req))
        assert abs(res[req.rid].E - E) <= 1e-10 * max(1.0, abs(E)), req
    print(f"[serve] {len(trace)} requests, {srv.stats['steps']} steps")


@pytest.mark.parametrize("L,k,T", [(8, 4, 0.6), (16, 1, 0.3)])
def test_small_request_matches_oracle(mods, L, k, T):
    """A served request against the oracle from the identical initial state: the
    served lattice's Philox initial state equals the single-lattice one, exported from
    the device (the host and device logarithms of Box-Muller may differ by an ulp, so
    the oracle takes the device's couplings); same Philox draws."""
    hsg, B, S = mods
    seed, sweeps = 77 + L, 12
    req = S.Request(rid=0, seed=seed, L=L, T=T, sweeps=sweeps, k=k)
    res = S.Server(hbm_budget=16 << 20, n_slots=2, step_sweeps=5).run([req], realtime=False)[0]
    s0, J0 = (t.cpu().numpy() for t in hsg.Lattice(L, torch.float32, seed=seed).export())
    s = s0.copy()
    taint = np.zeros(L ** 3, dtype=np.uint8)
    r = O.sweep(L, seed, s, J0, T=T, k=k, n_sweeps=sweeps, E=O.energy(L, s0, J0), taint=taint)
    m = s.astype(np.float64).mean(axis=1)
    print(f"[serve] L={L} k={k}: E served={res.E:.9f} oracle={r['E']:.9f} "
          f"flagged={r['n_flagged']}", flush=True)
    assert not taint.any()
    assert abs(res.E - r["E"]) <= 1e-5 * abs(r["E"])
    np.testing.assert_allclose(res.m, m, rtol=0, atol=1e-5)


def test_admission_waits_for_memory(mods):
    hsg, B, S = mods
    # 4 lattices of L=32 need 4 * 2 * 3 * 32^3 * 4 B = 3.1 MB; a 1.6 MB budget holds 2
    trace = [S.Request(rid=r, seed=9 + r, L=32, T=0.5, sweeps=20, k=1) for r in range(4)]
    srv = S.Server(hbm_budget=1_600_000, n_slots=8, step_sweeps=10)
    res = srv.run(trace, realtime=False)
    assert sorted(r.rid for r in res) == [0, 1, 2, 3]
    assert srv.arena_s.used == 0 and srv.arena_j.used == 0 and not srv.active
    # the budget holds two: the later two were admitted only once one of the first two
    # had finished and released its memory (scheduler iterations)
    adm = {r.rid: r.admitted_step for r in res}
    fin = {r.rid: r.finished_step for r in res}
    print(f"[serve] admitted at {adm}, finished at {fin}", flush=True)
    assert adm[0] == adm[1] == 0
    assert min(adm[2], adm[3]) >= min(fin[0], fin[1]) > 0
    assert max(adm[2], adm[3]) >= max(fin[0], fin[1])
    assert srv.free_slots and len(srv.free_slots) == 8


def alone(S, req):
    return S.Server(hbm_budget=64 << 20, n_slots=4, step_sweeps=5).run([req], realtime=False)[0]


def test_unservable_requests_are_rejected_without_affecting_others(mods):
    """Requests that cannot be served (odd or too large L, no hit, T <= 0, a footprint
    over the budget) return at once with a reason; the others complete as if alone."""
    hsg, B, S = mods
    good = [S.Request(rid=r, seed=7000 + r, L=L, T=0.6, sweeps=20, k=k)
            for r, (L, k) in enumerate([(8, 1), (16, 4), (32, 1)])]
    bad = [S.Request(rid=10, seed=1, L=9, T=0.5, sweeps=5, k=1),
           S.Request(rid=11, seed=1, L=B.BATCH_L_MAX + 2, T=0.5, sweeps=5, k=1),
           S.Request(rid=12, seed=1, L=8, T=0.5, sweeps=5, k=0),
           S.Request(rid=13, seed=1, L=8, T=0.0, sweeps=5, k=1),
           S.Request(rid=14, seed=1, L=96, T=0.5, sweeps=5, k=1)]  # beyond a 4 MB budget
    trace = [bad[0], good[0], bad[1], bad[2], good[1], bad[3], bad[4], good[2]]
    res = {r.rid: r for r in S.Server(hbm_budget=4 << 20, n_slots=8, step_sweeps=6).run(
        trace, realtime=False)}
    assert sorted(res) == sorted(r.rid for r in trace)
    for r in bad:
        print(f"[serve] rid={r.rid}: {res[r.rid].status}")
        assert res[r.rid].status.startswith("rejected: ") and math.isnan(res[r.rid].E)
        assert res[r.rid].sweeps_done == -1
    for r in good:
        a, b = alone(S, r), res[r.rid]
        assert b.status == "ok" and b.sweeps_done == r.sweeps
        np.testing.assert_array_equal(a.m, b.m)
        assert abs(a.E - b.E) <= 1e-12 * max(1.0, abs(a.E))


def test_cancel_resident_and_queued_requests(mods):
    """cancel() from the iteration hook: a resident long request stops and returns the
    state after the sweeps it made (equal to an alone run of that many sweeps); a queued
    one returns at once, never admitted; the others are unaffected."""
    hsg, B, S = mods
    long = S.Request(rid=0, seed=8100, L=32, T=0.4, sweeps=100000, k=4)
    short = [S.Request(rid=r, seed=8100 + r, L=16, T=0.7, sweeps=30, k=1) for r in (1, 2)]
    queued = S.Request(rid=3, seed=8200, L=16, T=0.7, sweeps=30, k=1)
    srv = S.Server(hbm_budget=64 << 20, n_slots=3, step_sweeps=4)  # queued waits for a slot

    def hook(it, server):
        if it == 2:
            server.cancel(0)
            server.cancel(3)
            server.cancel(12345)  # unknown: ignored

    res = {r.rid: r for r in srv.run([long, *short, queued], realtime=False, on_iteration=hook)}
    assert sorted(res) == [0, 1, 2, 3]
    c = res[0]
    print(f"[serve] cancelled after {c.sweeps_done} sweeps, E={c.E:.6f}")
    assert c.status == "cancelled" and 0 < c.sweeps_done < long.sweeps
    a = alone(S, S.Request(rid=0, seed=long.seed, L=long.L, T=long.T, sweeps=c.sweeps_done,
                           k=long.k))
    np.testing.assert_array_equal(a.m, c.m)
    assert abs(a.E - c.E) <= 1e-12 * max(1.0, abs(a.E))
    q = res[3]
    assert q.status == "cancelled" and q.sweeps_done == -1 and math.isnan(q.E)
    for r in short:
        assert res[r.rid].status == "ok" and res[r.rid].sweeps_done == r.sweeps
        np.testing.assert_array_equal(alone(S, r).m, res[r.rid].m)
    assert len(srv.free_slots) == 3 and not srv.active


def test_pass_sweep_equals_chain_sweep(mods):
    hsg, B, S = mods
    specs = [B.ChainSpec(L=L, seed=300 + i, J_group=i, J_seed=400 + i, T=0.4 + 0.1 * i, k=k,
                         n_or=1, renorm_every=3)
             for i, (L, k) in enumerate([(8, 1), (16, 4), (24, 2), (64, 4), (96, 1)])]
    a = B.Batch(specs, track_remaining=True)
    b = B.Batch(specs, track_remaining=True)
    budget = torch.tensor([5, 7, 3, 7, 6], dtype=torch.int32)
    a.remaining.copy_(budget)
    b.remaining.copy_(budget)
    a.sweep(7)
    table = b.table
    act = np.arange(len(specs), dtype=np.int32)
    import ctypes
    cap = 4096
    tiles = np.zeros(2 * cap, dtype=np.int32)
    n = ctypes.c_int32()
    hsg.check(hsg.lib().hsg_batch_tiles(table.ctypes.data_as(ctypes.c_void_p), len(specs),
                                        act.ctypes.data_as(ctypes.c_void_p), act.size, 256,
                                        tiles.ctypes.data_as(ctypes.c_void_p), cap,
                                        ctypes.byref(n)))
    td = torch.from_numpy(tiles[:2 * n.value].copy()).cuda()
    hsg.check(hsg.lib().hsg_batch_pass_sweep(ctypes.byref(b._d), hsg._ptr(td), n.value, 256, 1, 1,
                                             7, hsg._stream(None)))
    torch.cuda.synchronize()
    assert torch.equal(a.spins, b.spins)
    assert torch.equal(a.sweep_ctr, b.sweep_ctr) and torch.equal(a.remaining, b.remaining)
    assert torch.allclose(a.E, b.E, rtol=1e-12, atol=0)
