"""Serving engine: continuous batching must not change any result.  A request
scored alone, scored in a busy mix of other requests (other sizes and grid
sizes, several slots in flight), and scored by cf_score_poses directly give
bitwise the same scores; scores also meet the oracle bound."""
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import BF16_PK_TOL, weights

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"\n[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    from paper_2104_04547_amd.serve import Engine
    arch, w = weights("full")
    pool = synth.make_poses("c5", 96)
    eng = Engine(arch, w, "bf16", n_slots=3, slot_poses=128, slot_atoms=128 * 1600, hbm_budget_bytes=24 << 30)
    yield arch, w, pool, eng
    eng.close()


def test_alone_equals_in_the_mix_equals_direct(setup):
    import torch
    from paper_2104_04547_amd import Scorer, cfabi
    arch, w, pool, eng = setup
    target = pool.select(list(range(5, 12)))
    _say("engine: request alone, G=48")
    alone, lat = eng.result(eng.submit(target, 48), target.n_poses)
    assert lat > 0
    _say("engine: same request inside a mix of 24 requests, G in {48, 32}")
    rng = np.random.default_rng(0)
    tickets = []
    for i in range(24):
        if i == 11:
            tickets.append(("t", eng.submit(target, 48), target.n_poses))
        k = int(rng.integers(1, 40))
        sub = pool.select([int(j) for j in rng.integers(0, pool.n_poses, size=k)])
        tickets.append(("o", eng.submit(sub, int(rng.choice([48, 32]))), k))
    mixed = None
    for kind, t, n in tickets:
        s, _ = eng.result(t, n)
        if kind == "t":
            mixed = s
    assert np.array_equal(alone, mixed)
    _say("cf_score_poses on the same poses")
    sc = Scorer(arch, w, "bf16")
    try:
        direct = sc.score(cfabi.DeviceBatch.from_pose_batch(target), 48).cpu().numpy()
        sc.check()
    finally:
        sc.close()
    assert np.array_equal(alone, direct)
    info = eng.info()
    assert info["batches"] >= 2 and info["graph_replays"] >= 2


def test_graphs_survive_scratch_growth():
    # a graph captured for a small batch must not be replayed after a larger
    # batch has made the slot's context reallocate its scratch: the engine drops
    # and re-captures it, and the result stays bitwise the same
    from paper_2104_04547_amd import Scorer, cfabi
    from paper_2104_04547_amd.serve import Engine
    arch, w = weights("full")
    pool = synth.make_poses("c5", 80)
    small = pool.select(list(range(3)))
    big = pool.select(list(range(3, 80)))
    eng = Engine(arch, w, "bf16", n_slots=1, slot_poses=128, slot_atoms=128 * 1600, hbm_budget_bytes=16 << 30)
    try:
        _say("engine: small batch at G=32 (graph captured)")
        first, _ = eng.result(eng.submit(small, 32), 3)
        _say("engine: 77 poses at G=64 (scratch grows)")
        eng.result(eng.submit(big, 64), big.n_poses)
        _say("engine: small batch at G=32 again (graph captured again)")
        again, _ = eng.result(eng.submit(small, 32), 3)
    finally:
        eng.close()
    assert np.array_equal(first, again)
    sc = Scorer(arch, w, "bf16")
    try:
        direct = sc.score(cfabi.DeviceBatch.from_pose_batch(small), 32).cpu().numpy()
        sc.check()
    finally:
        sc.close()
    assert np.array_equal(first, direct)


def test_engine_scores_meet_the_oracle_bound(setup):
    arch, w, pool, eng = setup
    sub = pool.select([0, 1])
    _say("engine vs oracle, 2 poses, G=32")
    got, _ = eng.result(eng.submit(sub, 32), 2)
    for p in range(2):
        a, b = int(sub.atom_off[p]), int(sub.atom_off[p + 1])
        want = oracle.score_pose(sub.xyz[a:b], sub.feat[a:b], sub.is_lig[a:b], w, arch, 32)
        assert abs(float(got[p]) - want) <= BF16_PK_TOL


def test_engine_rejects_malformed_requests_on_the_host(setup):
    from paper_2104_04547_amd import cfabi
    arch, w, pool, eng = setup
    b = pool.select([0, 1])
    bad = synth.PoseBatch(np.array([0, 0, b.atom_off[2]], np.int32), b.xyz, b.feat, b.is_lig, b.n_lig)
    with pytest.raises(cfabi.CfError):
        eng.submit(bad, 48)            # empty pose
    with pytest.raises(cfabi.CfError):
        eng.submit(b, 50)              # grid size not a multiple of 4


def test_engine_rejects_bad_features_on_the_host(setup):
    from paper_2104_04547_amd import cfabi
    arch, w, pool, eng = setup
    b = pool.select([0, 1])
    for bad_value in (np.nan, np.inf, 64.5):
        f = b.feat.copy()
        f[3, 14] = bad_value
        bad = synth.PoseBatch(b.atom_off, b.xyz, f, b.is_lig, b.n_lig)
        with pytest.raises(cfabi.CfError):
            eng.submit(bad, 48)


def _dense_pose(pool, n_side=11):
    """n_side^3 atoms on a 0.25 A lattice: every pair lies within 4.5 A, so its
    non-covalent list alone (n (n - 1) edges) exceeds a small slot's edge capacity."""
    g = np.arange(n_side) * 256
    xyz = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(np.int32) + 50000
    n = xyz.shape[0]
    feat = pool.feat[np.arange(n) % pool.n_atoms].copy()
    lig = np.zeros(n, np.uint8)
    lig[:40] = 1
    feat[:, 18] = np.where(lig == 1, 1.0, -1.0)
    return synth.PoseBatch(np.array([0, n], np.int32), xyz, feat, lig, np.array([40], np.int32))


def test_a_request_that_fails_on_the_device_fails_alone():
    # one request whose neighbour lists overflow the batch's edge capacity shares
    # a batch with good requests: only it reports the error, and the others get
    # bitwise the scores cf_score_poses gives them alone
    from paper_2104_04547_amd import Scorer, cfabi
    from paper_2104_04547_amd.serve import Engine
    arch, w = weights("full")
    pool = synth.make_poses("c1", 25)
    dense = _dense_pose(pool)
    assert dense.n_atoms * (dense.n_atoms - 1) > 16384 * 96
    eng = Engine(arch, w, "bf16", n_slots=1, slot_poses=16, slot_atoms=16384, hbm_budget_bytes=8 << 30,
                 use_graphs=False)
    goods = [pool.select(list(range(0, 4))), pool.select(list(range(4, 9)))]
    try:
        _say("engine: 16 poses at G=96 occupy the only slot")
        first = eng.submit(pool.select(list(range(9, 25))), 96)
        _say("engine: good, dense (1331 atoms on a 0.25 A lattice), good requests at G=24")
        t = [eng.submit(goods[0], 24), eng.submit(dense, 24), eng.submit(goods[1], 24)]
        eng.result(first, 16)
        got0, _ = eng.result(t[0], goods[0].n_poses)
        with pytest.raises(cfabi.CfError) as ei:
            eng.result(t[1], 1)
        assert ei.value.code == cfabi.CF_ERR_CAPACITY
        got2, _ = eng.result(t[2], goods[1].n_poses)
        info = eng.info()
    finally:
        eng.close()
    assert info["batches"] == 2   # the three requests did share one batch
    sc = Scorer(arch, w, "bf16")
    try:
        for sub, got in ((goods[0], got0), (goods[1], got2)):
            _say(f"cf_score_poses on {sub.n_poses} poses alone")
            direct = sc.score(cfabi.DeviceBatch.from_pose_batch(sub), 24).cpu().numpy()
            sc.check()
            assert np.array_equal(got, direct)
    finally:
        sc.close()


def test_cancel_a_queued_request():
    from paper_2104_04547_amd import cfabi
    from paper_2104_04547_amd.serve import Engine
    arch, w = weights("full")
    pool = synth.make_poses("c5", 70)
    eng = Engine(arch, w, "bf16", n_slots=1, slot_poses=64, slot_atoms=64 * 1600, hbm_budget_bytes=8 << 30,
                 use_graphs=False)
    try:
        _say("engine: 64 poses at G=64 occupy the only slot; three requests queue behind it")
        busy = eng.submit(pool.select(list(range(64))), 64)
        subs = [pool.select([64, 65]), pool.select([66, 67]), pool.select([68, 69])]
        t = [eng.submit(s, 32) for s in subs]
        assert eng.cancel(t[1])          # still queued
        assert not eng.cancel(t[1])      # already withdrawn
        eng.result(busy, 64)
        got0, _ = eng.result(t[0], 2)
        with pytest.raises(cfabi.CfError) as ei:
            eng.result(t[1], 2)
        assert ei.value.code == cfabi.CF_ERR_CANCELLED
        got2, _ = eng.result(t[2], 2)
        with pytest.raises(cfabi.CfError):
            eng.cancel(t[1])             # ticket released by the poll that reported it
        _say("engine: the same two requests again, nothing cancelled")
        again0, _ = eng.result(eng.submit(subs[0], 32), 2)
        again2, _ = eng.result(eng.submit(subs[2], 32), 2)
        info = eng.info()
    finally:
        eng.close()
    assert np.array_equal(got0, again0) and np.array_equal(got2, again2)
    assert info["poses_done"] == 64 + 2 + 2 + 2 + 2 and info["queued_poses"] == 0
