"""Pins for the oracle's 3D-CNN, spatial graph, SG-CNN and fusion head (CPU only).

References used here are independent of the oracle's code: torch's float64 CPU
conv3d / GRUCell / SELU, scipy's k-d tree, dense adjacency products, brute-force
pair loops, symmetry and invariance properties, and closed forms.
"""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
import synth


# ---------------------------------------------------------------- conv3d / CNN

@pytest.mark.parametrize("C,O,k,s,D", [(3, 4, 3, 1, 6), (5, 2, 5, 2, 9), (19, 6, 7, 2, 12), (4, 3, 7, 1, 5),
                                       (6, 5, 3, 2, 8), (19, 4, 5, 2, 10)])
def test_conv3d_matches_torch_float64(C, O, k, s, D):
    rng = np.random.default_rng(C * 100 + k)
    x = rng.standard_normal((C, D, D + 1, D + 2))
    w = rng.standard_normal((O, C, k, k, k))
    b = rng.standard_normal(O)
    got = oracle.conv3d(x, w, b, s)
    want = F.conv3d(torch.from_numpy(x)[None], torch.from_numpy(w), torch.from_numpy(b),
                    stride=s, padding=(k - 1) // 2)[0].numpy()
    assert got.shape == want.shape
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12)


def test_conv3d_delta_input_returns_flipped_kernel_cross_correlation():
    # A unit impulse at position q gives out[o, q - t + p] = w[o, 0, t] (cross-correlation).
    k, D = 5, 9
    w = np.arange(2 * 1 * k ** 3, dtype=np.float64).reshape(2, 1, k, k, k)
    x = np.zeros((1, D, D, D))
    q = 4
    x[0, q, q, q] = 1.0
    out = oracle.conv3d(x, w, np.zeros(2), 1)
    p = (k - 1) // 2
    for t0 in range(k):
        for t1 in range(k):
            for t2 in range(k):
                assert out[1, q - t0 + p, q - t1 + p, q - t2 + p] == w[1, 0, t0, t1, t2]


def test_conv3d_linear():
    rng = np.random.default_rng(5)
    x1, x2 = rng.standard_normal((2, 3, 6, 6, 6))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    z = np.zeros(2)
    lhs = oracle.conv3d(2.0 * x1 - 3.0 * x2, w, z, 1)
    rhs = 2.0 * oracle.conv3d(x1, w, z, 1) - 3.0 * oracle.conv3d(x2, w, z, 1)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


def test_batchnorm_folding_equals_unfolded_conv_bn():
    # Folding gamma / sqrt(var + eps) into the weights and the shift into the bias is
    # exact algebra; the scorer relies on it.
    rng = np.random.default_rng(9)
    x = rng.standard_normal((4, 7, 7, 7))
    w = rng.standard_normal((3, 4, 3, 3, 3))
    b = rng.standard_normal(3)
    g, bt, mu = rng.uniform(0.8, 1.2, 3), rng.normal(0, 0.05, 3), rng.normal(0, 0.05, 3)
    var = rng.uniform(0.8, 1.2, 3)
    unfolded = oracle.batchnorm(oracle.conv3d(x, w, b, 1), g, bt, mu, var)
    sc = g / np.sqrt(var + 1e-5)
    folded = oracle.conv3d(x, w * sc[:, None, None, None, None], (b - mu) * sc + bt, 1)
    np.testing.assert_allclose(folded, unfolded, rtol=1e-12, atol=1e-12)


class _TorchCNN(torch.nn.Module):
    """float64 torch model with the same structure, built from torch layers."""

    def __init__(self, arch, w):
        super().__init__()
        self.arch = arch
        self.convs = torch.nn.ModuleList()
        self.bns = torch.nn.ModuleList()
        for i, (ci, co, k, s, r) in enumerate(arch.conv):
            c = torch.nn.Conv3d(ci, co, k, stride=s, padding=(k - 1) // 2).double()
            c.weight.data = torch.from_numpy(w[f"conv{i}.w"].astype(np.float64))
            c.bias.data = torch.from_numpy(w[f"conv{i}.b"].astype(np.float64))
            if arch.bn:
                bn = torch.nn.BatchNorm3d(co, eps=1e-5).double().eval()
                bn.weight.data = torch.from_numpy(w[f"bn{i}.gamma"].astype(np.float64))
                bn.bias.data = torch.from_numpy(w[f"bn{i}.beta"].astype(np.float64))
                bn.running_mean = torch.from_numpy(w[f"bn{i}.mean"].astype(np.float64))
                bn.running_var = torch.from_numpy(w[f"bn{i}.var"].astype(np.float64))
            else:
                bn = torch.nn.Identity()
            self.convs.append(c)
            self.bns.append(bn)
        self.dense = None
        layers, prev = [], arch.c_last
        for name in ("cnn_dense", "cnn_dense2"):
            width = getattr(arch, name)
            if width:
                lin = torch.nn.Linear(prev, width).double()
                lin.weight.data = torch.from_numpy(w[name + ".w"].astype(np.float64))
                lin.bias.data = torch.from_numpy(w[name + ".b"].astype(np.float64))
                layers += [lin, torch.nn.ReLU()]
                prev = width
        if layers:
            self.dense = torch.nn.Sequential(*layers)

    def forward(self, x):
        ts = [x]
        for i, (ci, co, k, s, r) in enumerate(self.arch.conv):
            y = self.bns[i](self.convs[i](ts[-1]))
            if r >= 0:
                y = y + ts[r]
            ts.append(torch.relu(y))
        pooled = torch.nn.functional.adaptive_avg_pool3d(ts[-1], 1).flatten(1)
        return self.dense(pooled) if self.dense is not None else pooled


@pytest.mark.parametrize("arch_name,G", [("tiny", 12), ("full", 16), ("paper", 16)])
def test_cnn3d_forward_matches_torch_model(arch_name, G):
    arch = synth.ARCHS[arch_name]
    w = synth.make_weights(arch)
    rng = np.random.default_rng(1)
    grid = np.abs(rng.standard_normal((G, G, G, 19))) * (rng.random((G, G, G, 19)) < 0.1)
    lat, _ = oracle.cnn3d_forward(grid, w, arch)
    with torch.no_grad():
        want = _TorchCNN(arch, w)(torch.from_numpy(np.moveaxis(grid, -1, 0))[None])[0].numpy()
    np.testing.assert_allclose(lat, want, rtol=1e-11, atol=1e-13)


# ---------------------------------------------------------------- graph

def _brute_pairs(X, r):
    n = len(X)
    out = []
    for i in range(n):
        for j in range(n):
            if i != j:
                d = [int(X[i][a]) - int(X[j][a]) for a in range(3)]
                if d[0] * d[0] + d[1] * d[1] + d[2] * d[2] <= r * r:
                    out.append((i, j))
    return out


def test_radius_graph_matches_python_pair_loop_with_ties():
    rng = np.random.default_rng(2)
    X = rng.integers(-3000, 3000, size=(40, 3))
    X[1] = X[0] + np.array([4608, 0, 0])       # exactly at the cutoff: included
    X[2] = X[0] + np.array([4609, 0, 0])       # just beyond
    X[3] = X[0] + np.array([3, 4, 0]) * 1000   # 5000 u
    rp, col = oracle.radius_graph_pose(X, 4608)
    got = [(i, int(c)) for i in range(len(X)) for c in col[rp[i]:rp[i + 1]]]
    assert got == _brute_pairs(X, 4608)
    assert (0, 1) in got and (0, 2) not in got


def test_radius_graph_matches_kdtree_and_invariants():
    from scipy.spatial import cKDTree
    b = synth.make_poses("c2", 1, pose0=2)
    X = b.xyz.astype(np.int64)
    for r in (1638, 4608):
        rp, col = oracle.radius_graph_pose(X, r)
        pairs = cKDTree(X.astype(np.float64)).query_pairs(r=r, output_type="set")
        want = sorted({(i, j) for i, j in pairs} | {(j, i) for i, j in pairs})
        got = [(i, int(c)) for i in range(len(X)) for c in col[rp[i]:rp[i + 1]]]
        assert got == want
        for i in range(len(X)):                              # columns ascending per row
            assert np.all(np.diff(col[rp[i]:rp[i + 1]]) > 0)
    # covalent edges are exactly the generator's ligand bonds: n_lig - 1 bonds of a tree
    rp_c, col_c = oracle.radius_graph_pose(X, 1638)
    nl = int(b.n_lig[0])
    assert rp_c[-1] == 2 * (nl - 1)
    assert np.all(rp_c[nl:] == rp_c[nl])                  # pocket atoms have no covalent edge
    rp_n, col_n = oracle.radius_graph_pose(X, 4608)
    cov = {(i, int(c)) for i in range(len(X)) for c in col_c[rp_c[i]:rp_c[i + 1]]}
    nc = {(i, int(c)) for i in range(len(X)) for c in col_n[rp_n[i]:rp_n[i + 1]]}
    assert cov <= nc


def test_radius_graph_batch_offsets_never_cross_poses():
    b = synth.make_poses("c1", 3)
    rp, col = oracle.radius_graph_batch(b, 4608)
    for p in range(3):
        a, e = int(b.atom_off[p]), int(b.atom_off[p + 1])
        seg = col[rp[a]:rp[e]]
        assert seg.min() >= a and seg.max() < e


# ---------------------------------------------------------------- SG-CNN

def test_gru_cell_matches_torch():
    rng = np.random.default_rng(4)
    H, n = 16, 9
    cell = torch.nn.GRUCell(H, H).double()
    m, h = rng.standard_normal((2, n, H))
    want = cell(torch.from_numpy(m), torch.from_numpy(h)).detach().numpy()
    got = oracle.gru_cell(m, h, cell.weight_ih.detach().numpy(), cell.weight_hh.detach().numpy(),
                          cell.bias_ih.detach().numpy(), cell.bias_hh.detach().numpy())
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-14)


def test_aggregate_equals_dense_adjacency_product():
    from oracle.cf_oracle import aggregate
    b = synth.make_poses("c1", 1)
    rp, col = oracle.radius_graph_pose(b.xyz, 4608)
    n = b.n_atoms
    A = np.zeros((n, n))
    for i in range(n):
        A[i, col[rp[i]:rp[i + 1]]] = 1.0
    h = np.random.default_rng(0).standard_normal((n, 16))
    np.testing.assert_allclose(aggregate(h, rp, col), A @ h, rtol=1e-13, atol=1e-13)


def _local_graphs(xyz, arch):
    return oracle.radius_graph_pose(xyz, arch.r_cov_u), oracle.radius_graph_pose(xyz, arch.r_nc_u)


@pytest.mark.parametrize("arch_name", ["tiny", "full", "paper"])
def test_sgcnn_invariant_to_atom_order(arch_name):
    arch = synth.ARCHS[arch_name]
    w = synth.make_weights(arch)
    b = synth.make_poses("c1", 1, pose0=4)
    s0 = oracle.sgcnn_pose(b.feat, b.is_lig, *_local_graphs(b.xyz, arch), w, arch)
    perm = np.random.default_rng(7).permutation(b.n_atoms)
    xyz, feat, lig = b.xyz[perm], b.feat[perm], b.is_lig[perm]
    s1 = oracle.sgcnn_pose(feat, lig, *_local_graphs(xyz, arch), w, arch)
    np.testing.assert_allclose(s1, s0, rtol=1e-12, atol=1e-12 * np.abs(s0).max())


def test_sgcnn_isolated_atom_follows_gru_with_zero_message():
    arch = synth.ARCHS["tiny"]
    w = synth.make_weights(arch)
    x = np.random.default_rng(1).standard_normal((1, 19))
    empty = (np.zeros(2, dtype=np.int64), np.zeros(0, dtype=np.int64))
    s, h = oracle.sgcnn_pose(x, np.array([1]), empty, empty, w, arch, return_h=True)
    H = arch.H
    with torch.no_grad():
        ht = torch.from_numpy(x) @ torch.from_numpy(w["sg.embed.w"].astype(np.float64)).T \
            + torch.from_numpy(w["sg.embed.b"].astype(np.float64))
        for stage in ("cov", "nc"):
            cell = torch.nn.GRUCell(H, H).double()
            cell.weight_ih.data = torch.from_numpy(w[f"sg.{stage}.gru.w_ih"].astype(np.float64))
            cell.weight_hh.data = torch.from_numpy(w[f"sg.{stage}.gru.w_hh"].astype(np.float64))
            cell.bias_ih.data = torch.from_numpy(w[f"sg.{stage}.gru.b_ih"].astype(np.float64))
            cell.bias_hh.data = torch.from_numpy(w[f"sg.{stage}.gru.b_hh"].astype(np.float64))
            ht = cell(torch.zeros(1, H, dtype=torch.float64), ht)
        gate = torch.sigmoid(torch.cat([ht, torch.from_numpy(x)], 1)
                             @ torch.from_numpy(w["sg.gate.w"].astype(np.float64)).T
                             + torch.from_numpy(w["sg.gate.b"].astype(np.float64)))
        val = ht @ torch.from_numpy(w["sg.val.w"].astype(np.float64)).T \
            + torch.from_numpy(w["sg.val.b"].astype(np.float64))
    np.testing.assert_allclose(h, ht.numpy(), rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(s, (gate * val)[0].numpy(), rtol=1e-13, atol=1e-14)


def test_sgcnn_readout_only_sees_ligand_atoms():
    # Pocket atoms farther from every ligand atom than the rounds can propagate
    # (K_c * r_cov + K_n * r_nc) cannot change the latent; flipping every atom to
    # "pocket" gives the zero vector.
    arch = synth.ARCHS["tiny"]
    w = synth.make_weights(arch)
    b = synth.make_poses("c2", 1, pose0=1)
    X = b.xyz.astype(np.int64)
    lig = b.is_lig.astype(bool)
    reach = arch.K_c * arch.r_cov_u + arch.K_n * arch.r_nc_u
    d2 = ((X[:, None, :] - X[None, lig, :]) ** 2).sum(-1).min(axis=1)
    far = (~lig) & (d2 > reach * reach)
    assert far.sum() > 10
    g = _local_graphs(b.xyz, arch)
    s0 = oracle.sgcnn_pose(b.feat, b.is_lig, *g, w, arch)
    f2 = b.feat.copy()
    f2[far] = np.random.default_rng(3).standard_normal((far.sum(), 19)).astype(np.float32)
    s1 = oracle.sgcnn_pose(f2, b.is_lig, *g, w, arch)
    assert np.array_equal(s0, s1)
    s2 = oracle.sgcnn_pose(b.feat, np.zeros_like(b.is_lig), *g, w, arch)
    assert np.all(s2 == 0.0)


# ---------------------------------------------------------------- fusion

def test_selu_matches_torch_and_closed_form():
    x = np.array([-50.0, -3.0, -1.0, -1e-3, 0.0, 1e-3, 1.0, 7.5])
    want = F.selu(torch.from_numpy(x)).numpy()
    np.testing.assert_allclose(oracle.selu(x), want, rtol=1e-15, atol=1e-15)
    assert oracle.selu(np.array([1.0]))[0] == pytest.approx(1.0507009873554805, rel=1e-15)
    assert oracle.selu(np.array([-700.0]))[0] == pytest.approx(-1.0507009873554805 * 1.6732632423543772, rel=1e-15)


def test_fusion_head_hand_inputs():
    arch = synth.ARCHS["full"]
    w = {"fusion.hidden.w": np.eye(64, 74, dtype=np.float32) * 2.0,
         "fusion.hidden.b": np.full(64, -1.0, dtype=np.float32),
         "fusion.out.w": np.ones((1, 64), dtype=np.float32),
         "fusion.out.b": np.array([0.5], dtype=np.float32)}
    cnn = np.array([1.0] * 10)
    sg = np.zeros(64)
    # hidden = 2*z - 1: ten units at 1 -> selu(1) = lambda; 54 units at -1 -> lambda*alpha*(e^-1 - 1)
    lam, alp = 1.0507009873554805, 1.6732632423543772
    want = 10 * lam + 54 * lam * alp * (math.exp(-1.0) - 1.0) + 0.5
    assert oracle.fusion_head(cnn, sg, w, arch) == pytest.approx(want, rel=1e-14)
    tiny = synth.ARCHS["tiny"]
    wt = {"fusion.out.w": np.arange(32, dtype=np.float32)[None], "fusion.out.b": np.array([1.0], np.float32)}
    assert oracle.fusion_head(np.ones(16), np.ones(16), wt, tiny) == 1.0 + sum(range(32))


def test_late_fusion_is_mean():
    assert list(oracle.late_fusion(np.array([6.0, 8.0]), np.array([7.0, 4.0]))) == [6.5, 6.0]


def test_score_pose_composes_the_stages():
    arch = synth.ARCHS["tiny"]
    w = synth.make_weights(arch)
    b = synth.make_poses("c1", 1, pose0=9)
    s, d = oracle.score_pose(b.xyz, b.feat, b.is_lig, w, arch, 24, detail=True)
    cnn, _ = oracle.cnn3d_forward(oracle.splat_pose(b.xyz, b.feat, d["center"], 24), w, arch)
    sg = oracle.sgcnn_pose(b.feat, b.is_lig, *_local_graphs(b.xyz, arch), w, arch)
    assert s == oracle.fusion_head(cnn, sg, w, arch)


# ---------------------------------------------------------------- PotentialNet staging

def _staged(width, K_c=2, K_n=2):
    """Small staged / unstaged architecture pair with equal stage widths."""
    import dataclasses
    base = dataclasses.replace(synth.ARCHS["tiny"], name="t_unstaged", H=width, K_c=K_c, K_n=K_n)
    return base, dataclasses.replace(base, name="t_staged", H_nc=width)


def test_staged_sgcnn_with_pass_through_gather_is_the_unstaged_model():
    # gate 0 -> sigmoid = 1/2, value 2 I -> the covalent gather returns h exactly,
    # embedding I -> the non-covalent stage starts from h; with the second block of
    # the final gate zeroed in both models they compute the same function, so any
    # misplaced stage, gather or embedding shows up here
    unst, st = _staged(16)
    wu = synth.make_weights(unst)
    ws = dict(synth.make_weights(st))
    for k, v in wu.items():
        if k.startswith("sg.") and k in ws and ws[k].shape == v.shape:
            ws[k] = v
    H = 16
    ws["sg.mid.gate.w"] = np.zeros((H, H + 19), np.float32)
    ws["sg.mid.gate.b"] = np.zeros(H, np.float32)
    ws["sg.mid.val.w"] = (2 * np.eye(H)).astype(np.float32)
    ws["sg.mid.val.b"] = np.zeros(H, np.float32)
    ws["sg.embed2.w"] = np.eye(H, dtype=np.float32)
    ws["sg.embed2.b"] = np.zeros(H, np.float32)
    wu = dict(wu)
    wu["sg.gate.w"] = wu["sg.gate.w"].copy()
    wu["sg.gate.w"][:, H:] = 0.0
    ws["sg.gate.w"] = np.concatenate([wu["sg.gate.w"][:, :H], np.zeros((H, H), np.float32)], axis=1)
    b = synth.make_poses("c1", 1, pose0=2)
    su = oracle.sgcnn_pose(b.feat, b.is_lig, *_local_graphs(b.xyz, unst), wu, unst)
    ss = oracle.sgcnn_pose(b.feat, b.is_lig, *_local_graphs(b.xyz, st), ws, st)
    np.testing.assert_allclose(ss, su, rtol=1e-13, atol=1e-13)
    # and the gather matters once it is not a pass-through
    ws["sg.mid.val.b"] = np.full(H, 0.5, np.float32)
    s2 = oracle.sgcnn_pose(b.feat, b.is_lig, *_local_graphs(b.xyz, st), ws, st)
    assert np.abs(s2 - su).max() > 1e-6


def test_staged_sgcnn_is_unchanged_by_zero_padding_the_covalent_width():
    # padding the covalent stage from 24 to 32 features with zero weights and
    # biases leaves the latent unchanged (pad features stay exactly 0 through the
    # GRU: r = z = 1/2, n = tanh(0) = 0); the GPU path relies on this
    import dataclasses
    arch = synth.ARCHS["paper"]
    w = synth.make_weights(arch)
    P = 32
    H, N = arch.H, arch.H_nc
    wp = dict(w)

    def pad(a, rows=None, cols=None):
        a = np.asarray(a, np.float32)
        out = np.zeros((rows if rows else a.shape[0],) + ((cols,) if cols else a.shape[1:]), np.float32)
        out[tuple(slice(0, d) for d in a.shape)] = a
        return out

    def pad_gates(a, cols=None):   # [3H, ...] stacked gates r, z, n -> [3P, ...]
        parts = [pad(a[g * H:(g + 1) * H], P, cols) for g in range(3)]
        return np.concatenate(parts, axis=0)

    wp["sg.embed.w"] = pad(w["sg.embed.w"], P)
    wp["sg.embed.b"] = pad(w["sg.embed.b"], P)
    for t in range(arch.K_c):
        wp[f"sg.cov.msg{t}.w"] = pad(w[f"sg.cov.msg{t}.w"], P, P)
    wp["sg.cov.gru.w_ih"] = pad_gates(w["sg.cov.gru.w_ih"], P)
    wp["sg.cov.gru.w_hh"] = pad_gates(w["sg.cov.gru.w_hh"], P)
    wp["sg.cov.gru.b_ih"] = pad_gates(w["sg.cov.gru.b_ih"])
    wp["sg.cov.gru.b_hh"] = pad_gates(w["sg.cov.gru.b_hh"])
    g = w["sg.mid.gate.w"]
    gp = np.zeros((P, P + 19), np.float32)
    gp[:H, :H] = g[:, :H]
    gp[:H, P:] = g[:, H:]
    wp["sg.mid.gate.w"] = gp
    wp["sg.mid.gate.b"] = pad(w["sg.mid.gate.b"], P)
    wp["sg.mid.val.w"] = pad(w["sg.mid.val.w"], P, P)
    wp["sg.mid.val.b"] = pad(w["sg.mid.val.b"], P)
    wp["sg.embed2.w"] = pad(w["sg.embed2.w"], N, P)
    gg = w["sg.gate.w"]
    ggp = np.zeros((N, N + P), np.float32)
    ggp[:, :N] = gg[:, :N]
    ggp[:, N:N + H] = gg[:, N:]
    wp["sg.gate.w"] = ggp
    arch_p = dataclasses.replace(arch, H=P)
    b = synth.make_poses("c2", 1, pose0=1)
    s0 = oracle.sgcnn_pose(b.feat, b.is_lig, *_local_graphs(b.xyz, arch), w, arch)
    s1 = oracle.sgcnn_pose(b.feat, b.is_lig, *_local_graphs(b.xyz, arch_p), wp, arch_p)
    np.testing.assert_allclose(s1, s0, rtol=1e-12, atol=1e-12 * np.abs(s0).max())


def test_second_dense_layer_selecting_units_truncates_the_latent():
    # dense2 = [I | 0] with zero bias keeps the first units of the (non-negative)
    # first dense layer's output
    import dataclasses
    arch = synth.ARCHS["paper"]
    w = dict(synth.make_weights(arch))
    w["cnn_dense2.w"] = np.eye(arch.cnn_dense2, arch.cnn_dense, dtype=np.float32)
    w["cnn_dense2.b"] = np.zeros(arch.cnn_dense2, np.float32)
    rng = np.random.default_rng(4)
    grid = np.abs(rng.standard_normal((12, 12, 12, 19))) * (rng.random((12, 12, 12, 19)) < 0.2)
    lat2, _ = oracle.cnn3d_forward(grid, w, arch)
    lat1, _ = oracle.cnn3d_forward(grid, w, dataclasses.replace(arch, cnn_dense2=0))
    np.testing.assert_array_equal(lat2, lat1[:arch.cnn_dense2])
