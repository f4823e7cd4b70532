"""End-to-end parity of cf_score_poses against stored FP64 oracle scores, plus
batch invariance, determinism, ragged batches and error handling.

Plain form (float32): |s_gpu - s_oracle| <= 1e-4 * max(1, |s_oracle|) per pose.
Precision form (bfloat16 operands, float32 accumulation): |error| <= 2e-2 pK.
Stored oracle values come from tests/golden/make_golden.py, which calls only the
oracle.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import BF16_PK_TOL, golden, golden_scores, score_tol, weights

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"\n[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def scorers(torch_mod):
    from paper_2104_04547_amd import Scorer
    out = {}
    for name in ("tiny", "full"):
        arch, w = weights(name)
        for prec in ("fp32", "bf16"):
            out[(name, prec)] = Scorer(arch, w, prec)
    yield out
    for s in out.values():
        s.close()


def _db(b, center=None):
    from paper_2104_04547_amd import cfabi
    return cfabi.DeviceBatch.from_pose_batch(b, center)


def _score(s, b, G):
    out = s.score(_db(b), G).cpu().numpy().astype(np.float64)
    rc, _, _ = s.status()
    assert rc == 0, f"device status {rc}"
    return out


@pytest.mark.parametrize("cfg,arch_name,G,n", [("c1", "tiny", 24, 64), ("c2", "full", 48, 64),
                                               ("c4", "full", 32, 16), ("c4", "full", 48, 16),
                                               ("c4", "full", 64, 8), ("c2", "full", 40, 8)])
def test_score_fp32_matches_oracle(scorers, cfg, arch_name, G, n):
    gd = golden(cfg, G)
    if gd is None:
        pytest.skip(f"no stored oracle values for {cfg} G={G}")
    n = min(n, len(gd["poses"]))
    _say(f"cf_score_poses fp32 {cfg} G={G} poses={n}")
    b = synth.make_poses(cfg, n)
    want = np.array([p["score"] for p in gd["poses"][:n]])
    got = _score(scorers[(arch_name, "fp32")], b, G)
    err = np.abs(got - want)
    print(f"fp32 {cfg} G={G}: max |err| {err.max():.3e}  mean {err.mean():.3e}")
    assert np.all(err <= score_tol(want)), f"worst pose {int(err.argmax())}: {got[err.argmax()]} vs {want[err.argmax()]}"


@pytest.mark.parametrize("cfg,arch_name,G,n", [("c1", "tiny", 24, 64), ("c2", "full", 48, 64),
                                               ("c4", "full", 32, 16), ("c4", "full", 48, 16),
                                               ("c4", "full", 64, 8)])
def test_score_bf16_within_pk_bound(scorers, cfg, arch_name, G, n):
    gd = golden(cfg, G)
    if gd is None:
        pytest.skip(f"no stored oracle values for {cfg} G={G}")
    n = min(n, len(gd["poses"]))
    _say(f"cf_score_poses bf16 {cfg} G={G} poses={n}")
    b = synth.make_poses(cfg, n)
    want = np.array([p["score"] for p in gd["poses"][:n]])
    got = _score(scorers[(arch_name, "bf16")], b, G)
    err = np.abs(got - want)
    print(f"bf16 {cfg} G={G}: max |err| {err.max():.3e} pK  mean {err.mean():.3e} pK")
    assert err.max() <= BF16_PK_TOL


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_score_full_512_pose_chunk(scorers, prec):
    # one full 512-pose chunk at 48^3: the production launch shape (spectrum work
    # buffers of 2 x 1.7 GB, byte offsets past 2^31), every stored score compared
    want = golden_scores("c2", 48)
    if want is None or len(want) < 256:
        pytest.skip("no stored oracle scores for c2 G=48")
    n = 512
    _say(f"cf_score_poses {prec} c2 G=48 poses={n} (one chunk)")
    b = synth.make_poses("c2", n)
    got = _score(scorers[("full", prec)], b, 48)
    m = min(n, len(want))
    err = np.abs(got[:m] - want[:m])
    print(f"{prec} c2 G=48 {n}-pose chunk: {m} poses compared, max |err| {err.max():.3e}  mean {err.mean():.3e}")
    if prec == "fp32":
        assert np.all(err <= score_tol(want[:m])), f"worst pose {int(err.argmax())}"
    else:
        assert err.max() <= BF16_PK_TOL
    assert np.all(np.isfinite(got))


def test_score_stage_latents_match_oracle(scorers, torch_mod):
    # the latents that feed the fusion head, through the separate entry points
    _say("cf_voxelize -> cf_cnn3d_fwd, cf_build_graphs -> cf_sgcnn_fwd, c1 G=24 poses=8")
    gd = golden("c1", 24)
    b = synth.make_poses("c1", 8)
    s = scorers[("tiny", "fp32")]
    db = _db(b)
    grid = s.voxelize(db, 24)
    cnn = s.cnn3d(grid, 24).cpu().numpy()
    sg = s.sgcnn(db, s.build_graphs(db)).cpu().numpy()
    assert s.status()[0] == 0
    want_c = np.array([p["cnn_lat"] for p in gd["poses"][:8]])
    want_s = np.array([p["sg_lat"] for p in gd["poses"][:8]])
    np.testing.assert_allclose(cnn, want_c, rtol=1e-4, atol=1e-5 * np.abs(want_c).max())
    np.testing.assert_allclose(sg, want_s, rtol=1e-4, atol=1e-5 * np.abs(want_s).max())


def test_score_batch_invariance_and_determinism(scorers):
    _say("cf_score_poses alone vs in batch, c2 G=48")
    b = synth.make_poses("c2", 12)
    for prec in ("fp32", "bf16"):
        s = scorers[("full", prec)]
        full = _score(s, b, 48)
        again = _score(s, b, 48)
        assert np.array_equal(full, again)          # run to run: bitwise
        for p in (0, 5, 11):
            alone = _score(s, b.pose(p), 48)
            assert alone[0] == full[p]               # alone vs in a batch: bitwise
        mixed = _score(s, b.select([11, 3, 7]), 48)
        assert np.array_equal(mixed, full[[11, 3, 7]])


def test_score_ragged_batch_with_tiny_and_large_poses(scorers):
    # one single-atom pose, one pose entirely outside the grid, and large poses
    _say("cf_score_poses ragged edge poses, full G=32")
    arch, w = weights("full")
    b = synth.make_poses("c4", 6)
    one = synth.PoseBatch(np.array([0, 1], np.int32), b.xyz[:1].copy(), b.feat[:1].copy(),
                          np.ones(1, np.uint8), np.array([1], np.int32))
    far = b.pose(1)
    far.xyz = far.xyz + np.int32(200 * 1024)
    far_center = np.zeros((1, 3), np.int32)   # grid at the origin, atoms 200 A away
    s = scorers[("full", "fp32")]
    got_one = _score(s, one, 32)
    want_one = oracle.score_pose(one.xyz, one.feat, one.is_lig, w, arch, 32)
    assert abs(got_one[0] - want_one) <= 1e-4 * max(1.0, abs(want_one))
    got_far = s.score(_db(far, far_center), 32).cpu().numpy().astype(np.float64)
    assert s.status()[0] == 0
    want_far = oracle.score_pose(far.xyz, far.feat, far.is_lig, w, arch, 32, center=far_center[0])
    assert abs(got_far[0] - want_far) <= 1e-4 * max(1.0, abs(want_far))


def test_score_chunking_matches_single_launch(torch_mod):
    # a tiny HBM budget forces many chunks; results must equal the one-chunk run
    _say("cf_score_poses chunked (small budget) vs default, c1 G=24 poses=40")
    from paper_2104_04547_amd import Scorer
    arch, w = weights("tiny")
    b = synth.make_poses("c1", 40)
    s_big = Scorer(arch, w, "fp32")
    s_small = Scorer(arch, w, "fp32", hbm_budget_bytes=200 << 20)
    try:
        a = _score(s_big, b, 24)
        c = _score(s_small, b, 24)
        assert np.array_equal(a, c)
    finally:
        s_big.close()
        s_small.close()


def test_budget_holds_across_grid_sizes(torch_mod):
    # scratch held from a smaller grid (and from the atom stages) counts against
    # the budget when a larger grid is tuned and scored: the chunk shrinks instead
    # of the call failing, and the scores still meet the oracle bound
    _say("budget across grid sizes: c4 G=32 then autotune + score at G=64, 1.5 GiB budget")
    from paper_2104_04547_amd import Scorer
    arch, w = weights("full")
    g64 = golden("c4", 64)
    n = len(g64["poses"])
    b = synth.make_poses("c4", 16)
    s = Scorer(arch, w, "bf16", hbm_budget_bytes=3 << 29)
    try:
        _score(s, b, 32)
        s.autotune(64, 512)
        got = _score(s, b.select(list(range(n))), 64)
    finally:
        s.close()
    want = np.array([p["score"] for p in g64["poses"]])
    assert np.abs(got - want).max() <= BF16_PK_TOL


def test_score_rejects_bad_arguments(scorers):
    _say("host-side argument checks")
    from paper_2104_04547_amd import cfabi
    s = scorers[("tiny", "fp32")]
    b = synth.make_poses("c1", 2)
    db = _db(b)
    with pytest.raises(cfabi.CfError) as e:
        s.score(db, 26)                      # not a multiple of 4
    assert e.value.code == cfabi.CF_ERR_UNSUPPORTED
    bad = cfabi.cf_pose_batch(0, db.n_atoms, db.atom_off.data_ptr(), db.xyz.data_ptr(), db.feat.data_ptr(),
                              db.is_lig.data_ptr(), None)
    import torch
    out = torch.empty(2, device="cuda")
    with pytest.raises(cfabi.CfError) as e:
        cfabi.cf_score_poses(s.ctx, bad, 24, out.data_ptr(), cfabi.current_stream())
    assert e.value.code == cfabi.CF_ERR_INVALID_ARG


def test_score_device_reports_bad_features(scorers):
    _say("device-side feature check (NaN feature)")
    from paper_2104_04547_amd import cfabi
    s = scorers[("tiny", "fp32")]
    b = synth.make_poses("c1", 2)
    b.feat[3, 14] = np.nan
    s.score(_db(b), 24)
    rc, _, _ = s.status()
    assert rc == cfabi.CF_ERR_INVALID_ARG
    assert s.status()[0] == 0                # the status word was cleared


def test_score_with_roctx_ranges_and_timing_unchanged(scorers):
    # stage ranges for a tracer and per-launch event timing only observe: the
    # scores are bitwise those of a plain call
    from paper_2104_04547_amd import cfabi
    _say("cf_score_poses bf16 c2 G=48 poses=8 with CF_TIMING_ROCTX | CF_TIMING_EVENTS")
    s = scorers[("full", "bf16")]
    b = synth.make_poses("c2", 8)
    plain = _score(s, b, 48)
    cfabi.cf_timing_enable(s.ctx, True, roctx=True)
    try:
        traced = _score(s, b, 48)
        stats = cfabi.cf_timing_read(s.ctx)
    finally:
        cfabi.cf_timing_enable(s.ctx, False)
    assert np.array_equal(plain, traced)
    assert "splat" in stats and stats["splat"]["launches"] >= 1
