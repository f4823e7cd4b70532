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
