"""Pins for the oracle's backward pass (CPU only).

Coherent Fusion fine-tunes both branches through the fused head (Sec. 2.2,
Table V); the oracle's gradients (oracle/cf_grad.py) are checked against two
references that share nothing with its code:

* torch float64 autograd through models built here from torch ops (conv3d,
  BatchNorm written as its formula, ReLU, mean pool, Linear, GRUCell, SELU), with
  every parameter a leaf tensor;
* central finite differences of the oracle's own forward score, one entry of
  every parameter tensor of the tiny model (and a few of the full model), so a
  dropped term anywhere in the backward fails.
"""
import dataclasses

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
import synth
from test_oracle_sgcnn_ref import TorchSGCNN


def _leaf(a):
    return torch.tensor(np.asarray(a, np.float64), requires_grad=True)


# ---------------------------------------------------------------- single ops

@pytest.mark.parametrize("C,O,k,s,D", [(3, 4, 3, 1, 6), (5, 2, 5, 2, 9), (4, 3, 7, 1, 8), (6, 5, 7, 2, 11)])
def test_conv3d_vjp_matches_torch_autograd(C, O, k, s, D):
    rng = np.random.default_rng(C + 10 * k + s)
    x, w, b = rng.standard_normal((C, D, D + 1, D + 2)), rng.standard_normal((O, C, k, k, k)), rng.standard_normal(O)
    y = oracle.conv3d(x, w, b, s)
    dy = rng.standard_normal(y.shape)
    tx, tw, tb = _leaf(x), _leaf(w), _leaf(b)
    (F.conv3d(tx[None], tw, tb, stride=s, padding=(k - 1) // 2)[0] * torch.from_numpy(dy)).sum().backward()
    dx, dw, db = oracle.conv3d_vjp(x, w, s, dy)
    np.testing.assert_allclose(dx, tx.grad.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(dw, tw.grad.numpy(), rtol=1e-11, atol=1e-11)
    np.testing.assert_allclose(db, tb.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_batchnorm_vjp_matches_torch_autograd():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 5, 5, 5))
    g, bt, mu, v = rng.uniform(0.8, 1.2, 4), rng.normal(0, 0.1, 4), rng.normal(0, 0.1, 4), rng.uniform(0.8, 1.2, 4)
    dy = rng.standard_normal(x.shape)
    t = [_leaf(a) for a in (x, g, bt, mu, v)]
    sh = lambda a: a[:, None, None, None]
    y = sh(t[1]) * (t[0] - sh(t[3])) / torch.sqrt(sh(t[4]) + 1e-5) + sh(t[2])
    (y * torch.from_numpy(dy)).sum().backward()
    got = oracle.batchnorm_vjp(x, g, mu, v, dy)
    for a, ref in zip(got, (t[0], t[1], t[2], t[3], t[4])):
        np.testing.assert_allclose(a, ref.grad.numpy(), rtol=1e-11, atol=1e-12)


def test_gru_cell_vjp_matches_torch_grucell():
    rng = np.random.default_rng(4)
    n, H = 7, 5
    m, h = rng.standard_normal((n, H)), rng.standard_normal((n, H))
    wi, wh, bi, bh = (rng.standard_normal((3 * H, H)), rng.standard_normal((3 * H, H)),
                      rng.standard_normal(3 * H), rng.standard_normal(3 * H))
    dh_new = rng.standard_normal((n, H))
    cell = torch.nn.GRUCell(H, H).double()
    for p_, a in zip((cell.weight_ih, cell.weight_hh, cell.bias_ih, cell.bias_hh), (wi, wh, bi, bh)):
        p_.data = torch.from_numpy(a.copy())
    tm, th = _leaf(m), _leaf(h)
    (cell(tm, th) * torch.from_numpy(dh_new)).sum().backward()
    dm, dh, dwi, dwh, dbi, dbh = oracle.gru_cell_vjp(m, h, wi, wh, bi, bh, dh_new)
    for a, ref in ((dm, tm.grad), (dh, th.grad), (dwi, cell.weight_ih.grad), (dwh, cell.weight_hh.grad),
                   (dbi, cell.bias_ih.grad), (dbh, cell.bias_hh.grad)):
        np.testing.assert_allclose(a, ref.numpy(), rtol=1e-11, atol=1e-12)


def test_aggregate_vjp_is_the_transposed_adjacency():
    rng = np.random.default_rng(6)
    n, H = 9, 3
    A = (rng.random((n, n)) < 0.35) & ~np.eye(n, dtype=bool)   # not symmetric on purpose
    rp = np.concatenate([[0], np.cumsum(A.sum(1))])
    col = np.nonzero(A)[1]
    da = rng.standard_normal((n, H))
    np.testing.assert_allclose(oracle.aggregate_vjp(da, rp, col), A.T.astype(float) @ da, rtol=1e-14, atol=1e-14)


# ---------------------------------------------------------------- branches and head

def _torch_cnn(arch, w, grid):
    """3D-CNN latent from torch ops with every parameter a leaf (BatchNorm as its
    formula, so the running statistics get gradients too)."""
    P = {k: _leaf(v) for k, v in w.items() if k.startswith(("conv", "bn", "cnn_dense"))}
    ts = [torch.from_numpy(np.moveaxis(np.asarray(grid, np.float64), -1, 0))]
    sh = lambda a: a[:, None, None, None]
    for i, (ci, co, k, s, r) in enumerate(arch.conv):
        y = F.conv3d(ts[-1][None], P[f"conv{i}.w"], P[f"conv{i}.b"], stride=s, padding=(k - 1) // 2)[0]
        if arch.bn:
            y = sh(P[f"bn{i}.gamma"]) * (y - sh(P[f"bn{i}.mean"])) / torch.sqrt(sh(P[f"bn{i}.var"]) + 1e-5) \
                + sh(P[f"bn{i}.beta"])
        if r >= 0:
            y = y + ts[r]
        ts.append(torch.relu(y))
    lat = ts[-1].mean(dim=(1, 2, 3))
    for n in ("cnn_dense", "cnn_dense2"):
        if getattr(arch, n):
            lat = torch.relu(P[n + ".w"] @ lat + P[n + ".b"])
    return lat, P


@pytest.mark.parametrize("arch_name,G", [("tiny", 12), ("full", 12)])
def test_cnn3d_vjp_matches_torch_autograd(arch_name, G):
    arch = synth.ARCHS[arch_name]
    w = synth.make_weights(arch)
    b = synth.make_poses("c1", 1, pose0=2)
    grid = oracle.splat_pose(b.xyz, b.feat, oracle.pose_center(b.xyz[b.is_lig.astype(bool)]), G)
    lat, P = _torch_cnn(arch, w, grid)
    dlat = np.random.default_rng(3).standard_normal(lat.shape[0])
    (lat * torch.from_numpy(dlat)).sum().backward()
    got = oracle.cnn3d_vjp(grid, w, arch, dlat)
    assert set(got) == set(P)
    for k, t in P.items():
        ref = t.grad.numpy()
        np.testing.assert_allclose(got[k], ref, rtol=1e-9, atol=1e-12 * max(1.0, np.abs(ref).max()), err_msg=k)


_SG_NAMES = {"embed.weight": "sg.embed.w", "embed.bias": "sg.embed.b", "gru_c.weight_ih": "sg.cov.gru.w_ih",
             "gru_c.weight_hh": "sg.cov.gru.w_hh", "gru_c.bias_ih": "sg.cov.gru.b_ih", "gru_c.bias_hh": "sg.cov.gru.b_hh",
             "gru_n.weight_ih": "sg.nc.gru.w_ih", "gru_n.weight_hh": "sg.nc.gru.w_hh", "gru_n.bias_ih": "sg.nc.gru.b_ih",
             "gru_n.bias_hh": "sg.nc.gru.b_hh", "gate.weight": "sg.gate.w", "gate.bias": "sg.gate.b",
             "val.weight": "sg.val.w", "val.bias": "sg.val.b"}


def _sg_name(n):
    if n.startswith("msg_c."):
        return f"sg.cov.msg{n.split('.')[1]}.w"
    if n.startswith("msg_n."):
        return f"sg.nc.msg{n.split('.')[1]}.w"
    return _SG_NAMES[n]


@pytest.mark.parametrize("arch_name,cfg,pose", [("tiny", "c1", 3), ("full", "c2", 1), ("tiny_2x3", "c1", 5)])
def test_sgcnn_vjp_matches_torch_autograd(arch_name, cfg, pose):
    arch = (dataclasses.replace(synth.ARCHS["tiny"], name="tiny_2x3", K_c=2, K_n=3) if arch_name == "tiny_2x3"
            else synth.ARCHS[arch_name])
    w = synth.make_weights(arch)
    b = synth.make_poses(cfg, 1, pose0=pose)
    model = TorchSGCNN(arch, w)
    s, _ = model(b.xyz, b.feat, b.is_lig)
    ds = np.random.default_rng(8).standard_normal(s.shape[0])
    (s * torch.from_numpy(ds)).sum().backward()
    cov = oracle.radius_graph_pose(b.xyz, arch.r_cov_u)
    nc = oracle.radius_graph_pose(b.xyz, arch.r_nc_u)
    got = oracle.sgcnn_vjp(b.feat, b.is_lig, cov, nc, w, arch, ds)
    seen = set()
    for n, p_ in model.named_parameters():
        k = _sg_name(n)
        seen.add(k)
        ref = p_.grad.numpy()
        np.testing.assert_allclose(got[k], ref, rtol=1e-9, atol=1e-12 * max(1.0, np.abs(ref).max()), err_msg=k)
    assert seen == set(got)


@pytest.mark.parametrize("arch_name", ["tiny", "full", "full_res3"])
def test_fusion_head_vjp_matches_torch_autograd(arch_name):
    arch = (dataclasses.replace(synth.ARCHS["full"], name="full_res3", fusion_layers=4, fusion_residual=True)
            if arch_name == "full_res3" else synth.ARCHS[arch_name])
    w = synth.make_weights(arch)
    rng = np.random.default_rng(11)
    cnn, sg = rng.standard_normal(arch.cnn_latent), rng.standard_normal(arch.sg_latent)
    tc, ts = _leaf(cnn), _leaf(sg)
    P = {k: _leaf(v) for k, v in w.items() if k.startswith("fusion.")}
    z = torch.cat([tc, ts])
    for l in range(arch.n_fusion - 1):
        n = "fusion.hidden" if l == 0 else f"fusion.hidden{l}"
        y = F.selu(P[n + ".w"] @ z + P[n + ".b"])
        z = y + z if (arch.fusion_residual and l > 0) else y
    s = (P["fusion.out.w"] @ z + P["fusion.out.b"])[0]
    (2.5 * s).backward()
    dcnn, dsg, g = oracle.fusion_head_vjp(cnn, sg, w, arch, 2.5)
    np.testing.assert_allclose(dcnn, tc.grad.numpy(), rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(dsg, ts.grad.numpy(), rtol=1e-11, atol=1e-13)
    assert set(g) == set(P)
    for k, t in P.items():
        np.testing.assert_allclose(g[k], t.grad.numpy(), rtol=1e-11, atol=1e-13, err_msg=k)


# ---------------------------------------------------------------- whole score, finite differences

def _score_sum(b, w, arch, G, dscore):
    return sum(dscore[p] * oracle.score_pose(b.xyz[b.atom_off[p]:b.atom_off[p + 1]], b.feat[b.atom_off[p]:b.atom_off[p + 1]],
                                             b.is_lig[b.atom_off[p]:b.atom_off[p + 1]], w, arch, G)
               for p in range(b.n_poses))


def _fd_check(b, w, arch, G, dscore, names, rng, eps=1e-6):
    # a small step keeps ReLU kinks (a pre-activation within h of zero) out of most
    # difference quotients, and float64 round-off of the score (~1e-14 over its
    # thousands of terms) costs ~1e-14 / h; the bound is far below what a dropped
    # or misplaced term changes
    grads = oracle.score_vjp(b, w, arch, G, dscore)
    for k in names:
        flat = np.asarray(w[k], np.float64).ravel()
        idx = int(rng.integers(0, flat.size))
        g = np.asarray(grads[k]).ravel()[idx]
        h = eps * max(1.0, abs(flat[idx]))
        wp, wm = dict(w), dict(w)
        fp, fm = flat.copy(), flat.copy()
        fp[idx] += h
        fm[idx] -= h
        wp[k] = fp.reshape(np.shape(w[k]))
        wm[k] = fm.reshape(np.shape(w[k]))
        fd = (_score_sum(b, wp, arch, G, dscore) - _score_sum(b, wm, arch, G, dscore)) / (2 * h)
        assert abs(fd - g) <= 1e-4 * max(abs(fd), abs(g)) + 1e-7, f"{k}[{idx}]: vjp {g} vs finite difference {fd}"


def test_score_vjp_finite_differences_every_tiny_parameter():
    arch = synth.ARCHS["tiny"]
    w = {k: np.asarray(v, np.float64) for k, v in synth.make_weights(arch).items()}
    b = synth.make_poses("c1", 2, pose0=4)
    _fd_check(b, w, arch, 12, np.array([0.7, -1.3]), sorted(w), np.random.default_rng(21))


def test_score_vjp_finite_differences_full_model_sample():
    arch = synth.ARCHS["full"]
    w = {k: np.asarray(v, np.float64) for k, v in synth.make_weights(arch).items()}
    b = synth.make_poses("c1", 1, pose0=6)
    names = ["conv0.w", "bn2.var", "conv4.b", "conv5.w", "cnn_dense.w", "sg.cov.msg1.w", "sg.nc.gru.w_hh",
             "sg.gate.w", "fusion.hidden.w", "fusion.out.b"]
    _fd_check(b, w, arch, 8, np.array([1.0]), names, np.random.default_rng(22))


def test_score_vjp_is_linear_in_the_upstream_gradients():
    arch = synth.ARCHS["tiny"]
    w = synth.make_weights(arch)
    b = synth.make_poses("c1", 2, pose0=9)
    g1 = oracle.score_vjp(b, w, arch, 12, np.array([1.0, 0.0]))
    g2 = oracle.score_vjp(b, w, arch, 12, np.array([0.0, 1.0]))
    g = oracle.score_vjp(b, w, arch, 12, np.array([2.0, -3.0]))
    for k in g:
        np.testing.assert_allclose(g[k], 2.0 * g1[k] - 3.0 * g2[k], rtol=1e-10, atol=1e-13)
