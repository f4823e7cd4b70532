"""Per-stage parity of the HIP path (through the C ABI) against the FP64 oracle.

Integer stages (grid centres, neighbour lists) must match bit for bit; floating
point stages within tolerances derived from the arithmetic (float32 accumulation,
2^-20 fixed-point splat accumulators, bfloat16 operand rounding).
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import BF16_LATENT_TOL, weights

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


def _oracle_centers(b):
    return np.stack([oracle.pose_center(b.xyz[b.atom_off[p]:b.atom_off[p + 1]][b.is_lig[b.atom_off[p]:b.atom_off[p + 1]].astype(bool)])
                     for p in range(b.n_poses)])


# ------------------------------------------------------------------ centres

@pytest.mark.parametrize("cfg,n", [("c1", 64), ("c2", 32), ("c4", 40)])
def test_centers_bit_exact(scorers, cfg, n):
    _say(f"cf_pose_centers {cfg} poses={n}")
    b = synth.make_poses(cfg, n)
    got = scorers[("tiny", "fp32")].centers(_db(b)).cpu().numpy()
    assert np.array_equal(got, _oracle_centers(b))


def test_centers_pose_without_ligand_uses_all_atoms(scorers):
    _say("cf_pose_centers no-ligand pose")
    b = synth.make_poses("c1", 2)
    b.is_lig[b.atom_off[1]:b.atom_off[2]] = 0
    got = scorers[("tiny", "fp32")].centers(_db(b)).cpu().numpy()
    assert np.array_equal(got[1], oracle.pose_center(b.xyz[b.atom_off[1]:b.atom_off[2]]))


# ------------------------------------------------------------------ voxelisation

@pytest.mark.parametrize("cfg,n,G", [("c1", 16, 24), ("c2", 3, 48), ("c4", 4, 32)])
def test_voxelize_fp32_matches_oracle(scorers, cfg, n, G):
    _say(f"cf_voxelize fp32 {cfg} poses={n} G={G}")
    b = synth.make_poses(cfg, n)
    cen = _oracle_centers(b)
    got = scorers[("tiny", "fp32")].voxelize(_db(b, cen), G).cpu().numpy().astype(np.float64)
    want = oracle.splat_batch(b, cen, G)
    # per contribution: 2^-21 fixed-point rounding + float32 weight error (~1e-6 relative)
    np.testing.assert_allclose(got, want, rtol=2e-6, atol=1e-5)
    # mass bookkeeping: every channel sum agrees closely
    np.testing.assert_allclose(got.sum(axis=(1, 2, 3)), want.sum(axis=(1, 2, 3)), rtol=1e-5, atol=1e-3)


def test_voxelize_bf16_rounds_the_fp32_grid(scorers, torch_mod):
    _say("cf_voxelize bf16 c1 poses=8 G=24")
    b = synth.make_poses("c1", 8)
    cen = _oracle_centers(b)
    got = scorers[("tiny", "bf16")].voxelize(_db(b, cen), 24).float().cpu().numpy()
    want = oracle.splat_batch(b, cen, 24)
    np.testing.assert_allclose(got, want, rtol=2 ** -8, atol=1e-5)


def test_voxelize_exact_permutation_under_90deg_rotation(scorers):
    _say("cf_voxelize rotation c1 pose 1 G=24")
    b = synth.make_poses("c1", 1, pose0=1)
    c = _oracle_centers(b)
    d = b.xyz.astype(np.int64) - c[0]
    rot = b.pose(0)
    rot.xyz = (np.stack([-d[:, 1], d[:, 0], d[:, 2]], 1) + c[0]).astype(np.int32)
    s = scorers[("tiny", "fp32")]
    g = s.voxelize(_db(b, c), 24).cpu().numpy()
    gr = s.voxelize(_db(rot, c), 24).cpu().numpy()
    G = 24
    ii, jj, kk = np.meshgrid(np.arange(G), np.arange(G), np.arange(G), indexing="ij")
    want = np.empty_like(g[0])
    want[G - 1 - jj, ii, kk] = g[0][ii, jj, kk]
    # fixed-point accumulation makes the permuted grid agree to the last bit
    assert np.array_equal(gr[0], want)


def test_voxelize_is_deterministic(scorers):
    _say("cf_voxelize determinism c2 poses=2 G=48")
    b = synth.make_poses("c2", 2)
    s = scorers[("full", "fp32")]
    db = _db(b)
    a = s.voxelize(db, 48).cpu().numpy()
    c = s.voxelize(db, 48).cpu().numpy()
    assert np.array_equal(a, c)


def _coincident_pose(n):
    """n atoms on the centre of voxel (12, 12, 12) of a 24^3 grid centred on 0, |f| = 64."""
    rng = np.random.default_rng(n)
    F = (64.0 * rng.choice([-1.0, 1.0], size=(n, 19))).astype(np.float32)
    F[:, 0] = 64.0
    X = np.tile(np.array([[512, 512, 512]], np.int32), (n, 1))
    lig = np.zeros(n, np.uint8)
    lig[0] = 1
    b = synth.PoseBatch(np.array([0, n], np.int32), X, F, lig, np.array([1], np.int32))
    return b, np.zeros((1, 3), np.int64)


def test_voxelize_dense_pose_within_the_range_budget(scorers):
    # 60 coincident atoms at |f| = 64 use 3840 of a tile's 4096 budget: values up
    # to 60 * 64 * 0.492 = 1890 feature units, exact in the fixed-point accumulators
    _say("cf_voxelize 60 coincident atoms |f|=64 G=24")
    b, cen = _coincident_pose(60)
    s = scorers[("tiny", "fp32")]
    got = s.voxelize(_db(b, cen), 24).cpu().numpy().astype(np.float64)
    assert s.status()[0] == 0
    want = oracle.splat_batch(b, cen, 24)
    assert np.abs(want).max() > 1800.0
    np.testing.assert_allclose(got, want, rtol=2e-6, atol=1e-5)


def test_voxelize_reports_a_pose_beyond_the_range_budget(scorers):
    # 70 coincident atoms at |f| = 64: channel 0 of the centre voxel would reach
    # 70 * 64 * 0.492 = 2205 > 2048 feature units and wrap an int32 accumulator;
    # the tile's budget (4480 > 4096) reports it instead
    from paper_2104_04547_amd import cfabi
    _say("cf_voxelize 70 coincident atoms |f|=64 G=24 (reported)")
    b, cen = _coincident_pose(70)
    s = scorers[("tiny", "fp32")]
    s.voxelize(_db(b, cen), 24)
    assert s.status()[0] == cfabi.CF_ERR_INVALID_ARG
    assert "too dense" in cfabi.load().cf_last_error().decode()


# ------------------------------------------------------------------ neighbour lists

def _csr_host(t, n):
    import torch
    torch.cuda.synchronize()
    cr, nr = t["cov_row"].cpu().numpy(), t["nc_row"].cpu().numpy()
    return (cr, t["cov_col"].cpu().numpy()[:cr[n]]), (nr, t["nc_col"].cpu().numpy()[:nr[n]])


@pytest.mark.parametrize("cfg,n", [("c1", 64), ("c2", 8), ("c4", 24)])
def test_graphs_bit_exact(scorers, cfg, n):
    _say(f"cf_build_graphs {cfg} poses={n}")
    b = synth.make_poses(cfg, n)
    arch = synth.ARCHS["full"]
    s = scorers[("full", "fp32")]
    t = s.build_graphs(_db(b))
    rc, _, _ = s.status()
    assert rc == 0
    (cr, cc), (nr, ncol) = _csr_host(t, b.n_atoms)
    wr, wc = oracle.radius_graph_batch(b, arch.r_cov_u)
    assert np.array_equal(cr, wr) and np.array_equal(cc, wc)
    wr, wc = oracle.radius_graph_batch(b, arch.r_nc_u)
    assert np.array_equal(nr, wr) and np.array_equal(ncol, wc)


def test_graphs_ties_at_the_cutoff(scorers):
    _say("cf_build_graphs cutoff ties")
    # atoms exactly at r_nc / r_cov and one unit beyond
    x = np.array([[0, 0, 0], [4608, 0, 0], [0, 4609, 0], [0, 0, 1638], [1639, 0, 0], [0, -1638, 0]], np.int32)
    b = synth.PoseBatch(np.array([0, 6], np.int32), x, np.zeros((6, 19), np.float32), np.ones(6, np.uint8),
                        np.array([6], np.int32))
    s = scorers[("full", "fp32")]
    (cr, cc), (nr, ncol) = _csr_host(s.build_graphs(_db(b)), 6)
    wr, wc = oracle.radius_graph_pose(x, 1638)
    assert np.array_equal(cr, wr) and np.array_equal(cc, wc)
    wr, wc = oracle.radius_graph_pose(x, 4608)
    assert np.array_equal(nr, wr) and np.array_equal(ncol, wc)


def test_graphs_large_and_wide_poses(scorers):
    """A pose of more atoms than one j tile (1024) of the all-pairs sweep, a pose
    spanning more than 2^31 units on x (64-bit difference path) and a lone atom."""
    _say("cf_build_graphs 1500-atom pose, 2^31-wide pose, 1-atom pose")
    rng = np.random.default_rng(5)
    big = rng.integers(-16 * 1024, 16 * 1024, size=(1500, 3)).astype(np.int32)  # 32 A box
    wide = rng.integers(-3 * 1024, 3 * 1024, size=(60, 3)).astype(np.int64)
    wide[:30, 0] -= 1_100_000_000
    wide[30:, 0] += 1_100_000_000
    wide = wide.astype(np.int32)
    lone = np.array([[7, 8, 9]], np.int32)
    x = np.concatenate([big, wide, lone])
    off = np.array([0, 1500, 1560, 1561], np.int32)
    b = synth.PoseBatch(off, x, np.zeros((len(x), 19), np.float32), np.zeros(len(x), np.uint8),
                        np.array([0, 0, 0], np.int32))
    arch = synth.ARCHS["full"]
    s = scorers[("full", "fp32")]
    t = s.build_graphs(_db(b), cov_capacity=400_000, nc_capacity=2_000_000)
    rc, _, _ = s.status()
    assert rc == 0
    (cr, cc), (nr, ncol) = _csr_host(t, len(x))
    wr, wc = oracle.radius_graph_batch(b, arch.r_cov_u)
    assert np.array_equal(cr, wr) and np.array_equal(cc, wc)
    wr, wc = oracle.radius_graph_batch(b, arch.r_nc_u)
    assert np.array_equal(nr, wr) and np.array_equal(ncol, wc)


def test_graphs_capacity_overflow_reports_needed_counts(scorers):
    _say("cf_build_graphs capacity overflow")
    from paper_2104_04547_amd import cfabi
    b = synth.make_poses("c1", 4)
    s = scorers[("full", "fp32")]
    s.build_graphs(_db(b), cov_capacity=3, nc_capacity=10)
    rc, need_c, need_n = s.status()
    assert rc == cfabi.CF_ERR_CAPACITY
    wr, _ = oracle.radius_graph_batch(b, 1638)
    wn, _ = oracle.radius_graph_batch(b, 4608)
    assert need_c == wr[-1] and need_n == wn[-1]
    # a retry with the reported sizes succeeds
    s.build_graphs(_db(b), cov_capacity=need_c, nc_capacity=need_n)
    assert s.status()[0] == 0


def test_graphs_are_deterministic(scorers):
    _say("cf_build_graphs determinism c2 poses=4")
    b = synth.make_poses("c2", 4)
    s = scorers[("full", "fp32")]
    db = _db(b)
    a = _csr_host(s.build_graphs(db), b.n_atoms)
    c = _csr_host(s.build_graphs(db), b.n_atoms)
    for x, y in zip(a, c):
        assert np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1])


# ------------------------------------------------------------------ 3D-CNN

def _oracle_grids(b, G):
    return oracle.splat_batch(b, _oracle_centers(b), G)


@pytest.mark.parametrize("arch_name,cfg,n,G", [("tiny", "c1", 6, 24), ("full", "c1", 2, 24), ("full", "c2", 1, 40)])
def test_cnn3d_fp32_matches_oracle(scorers, torch_mod, arch_name, cfg, n, G):
    _say(f"cf_cnn3d_fwd fp32 arch={arch_name} {cfg} poses={n} G={G}")
    torch = torch_mod
    arch, w = weights(arch_name)
    b = synth.make_poses(cfg, n)
    grids = _oracle_grids(b, G)
    got = scorers[(arch_name, "fp32")].cnn3d(torch.from_numpy(grids.astype(np.float32)).cuda(), G).cpu().numpy()
    want = np.stack([oracle.cnn3d_forward(g, w, arch)[0] for g in grids])
    scale = np.abs(want).max(axis=1, keepdims=True) + 1e-6
    np.testing.assert_allclose(got, want, rtol=1e-4, atol=1e-4 * scale.max())


@pytest.mark.parametrize("arch_name,G", [("tiny", 24), ("full", 24)])
def test_cnn3d_bf16_within_operand_rounding(scorers, torch_mod, arch_name, G):
    _say(f"cf_cnn3d_fwd bf16 arch={arch_name} G={G}")
    torch = torch_mod
    arch, w = weights(arch_name)
    b = synth.make_poses("c1", 2)
    grids = _oracle_grids(b, G)
    got = scorers[(arch_name, "bf16")].cnn3d(torch.from_numpy(grids).to(torch.bfloat16).cuda(), G).cpu().numpy()
    want = np.stack([oracle.cnn3d_forward(g, w, arch)[0] for g in grids])
    scale = np.abs(want).max()
    np.testing.assert_allclose(got, want, rtol=BF16_LATENT_TOL, atol=BF16_LATENT_TOL * scale)


# ------------------------------------------------------------------ SG-CNN

def _oracle_csr_dev(b, arch, torch):
    from paper_2104_04547_amd import cfabi
    out = {}
    for key, r in (("cov", arch.r_cov_u), ("nc", arch.r_nc_u)):
        rp, col = oracle.radius_graph_batch(b, r)
        out[key + "_row"] = torch.from_numpy(rp.astype(np.int32)).cuda()
        col32 = col.astype(np.int32) if len(col) else np.zeros(1, np.int32)
        out[key + "_col"] = torch.from_numpy(col32).cuda()
        out[key] = cfabi.cf_csr(out[key + "_row"].data_ptr(), out[key + "_col"].data_ptr(), len(col))
    return out


@pytest.mark.parametrize("arch_name,cfg,n", [("tiny", "c1", 16), ("full", "c2", 4), ("full", "c4", 8)])
def test_sgcnn_fp32_matches_oracle(scorers, torch_mod, arch_name, cfg, n):
    _say(f"cf_sgcnn_fwd fp32 arch={arch_name} {cfg} poses={n}")
    arch, w = weights(arch_name)
    b = synth.make_poses(cfg, n)
    g = _oracle_csr_dev(b, arch, torch_mod)
    s = scorers[(arch_name, "fp32")]
    got = s.sgcnn(_db(b), g).cpu().numpy()
    assert s.status()[0] == 0
    want = oracle.sgcnn_batch(b, w, arch)
    scale = np.abs(want).max()
    np.testing.assert_allclose(got, want, rtol=1e-4, atol=2e-5 * scale)


def test_sgcnn_bf16_within_operand_rounding(scorers, torch_mod):
    _say("cf_sgcnn_fwd bf16 full c2 poses=4")
    arch, w = weights("full")
    b = synth.make_poses("c2", 4)
    g = _oracle_csr_dev(b, arch, torch_mod)
    got = scorers[("full", "bf16")].sgcnn(_db(b), g).cpu().numpy()
    want = oracle.sgcnn_batch(b, w, arch)
    scale = np.abs(want).max()
    # split (hi + lo) bfloat16 operands carry ~16 mantissa bits
    np.testing.assert_allclose(got, want, rtol=2e-3, atol=1e-3 * scale)


def test_sgcnn_atom_order_invariance(scorers, torch_mod):
    _say("cf_sgcnn_fwd atom permutation full c2 pose 0")
    arch, w = weights("full")
    b = synth.make_poses("c2", 1)
    perm = np.random.default_rng(5).permutation(b.n_atoms)
    bp = synth.PoseBatch(b.atom_off, b.xyz[perm], b.feat[perm], b.is_lig[perm], b.n_lig)
    s = scorers[("full", "fp32")]
    a = s.sgcnn(_db(b), _oracle_csr_dev(b, arch, torch_mod)).cpu().numpy()
    c = s.sgcnn(_db(bp), _oracle_csr_dev(bp, arch, torch_mod)).cpu().numpy()
    np.testing.assert_allclose(a, c, rtol=1e-4, atol=1e-5 * np.abs(a).max())
