"""FP64 CPU oracle of the backward pass: gradients of the Coherent Fusion score.

TEST INFRASTRUCTURE ONLY: the scoring library never imports this module and
shares no code with it.

Coherent Fusion is trained end to end: the fusion layers and both branches
(3D-CNN and SG-CNN) receive gradients through the concatenated latents, so the
whole model is fine-tuned together rather than its heads being trained apart
(Sec. 2.2; training hyper-parameters in Table V).  This module computes, for a
batch of poses and one upstream gradient per pose g_p = dL/ds_p (for a squared
error loss, s_p - y_p), the vector-Jacobian product

    grad[theta] = sum_p g_p * d s_p / d theta

for every parameter theta of the model blob (BatchNorm running mean and variance
included: at inference they are parameters of the function like any other).
Each function reverses one forward function of `cf_oracle`, step by step, from
the definitions written there; no step is fused or reordered.

Covered: the Coherent Fusion head (hidden SELU layers, optionally residual),
the 3D-CNN (conv, inference BatchNorm, ReLU, residual adds, mean pool, dense
layers) and the unstaged SG-CNN (embedding, gated rounds, gated ligand readout).
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

from .cf_oracle import (BN_EPS, SELU_ALPHA, SELU_LAMBDA, pose_center, radius_graph_pose, relu, selu, sigmoid,
                        splat_pose)


def _f64(w, k):
    return np.asarray(w[k], np.float64)


# --------------------------------------------------------------------------------
# 3D-CNN
# --------------------------------------------------------------------------------

def conv3d_vjp(x: np.ndarray, w: np.ndarray, stride: int, dy: np.ndarray):
    """Gradients of y = conv3d(x, w, b, stride) given dL/dy: (dx, dw, db).

    With zero padding p the forward reads x_pad[c, s*i + t] for every output i and
    tap t, so dL/dw[o, c, t] = sum_i dy[o, i] x_pad[c, s*i + t] and
    dL/dx_pad[c, s*i + t] += sum_o w[o, c, t] dy[o, i]; the padding is cut off
    dx_pad at the end.  x [C, D0, D1, D2], w [O, C, k, k, k], dy [O, o0, o1, o2]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    dy = np.asarray(dy, np.float64)
    C, D0, D1, D2 = x.shape
    O, k = w.shape[0], w.shape[2]
    p, s = (k - 1) // 2, stride
    o0, o1, o2 = dy.shape[1:]
    xp = np.zeros((C, D0 + 2 * p, D1 + 2 * p, D2 + 2 * p))
    xp[:, p:p + D0, p:p + D1, p:p + D2] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for t0 in range(k):
        for t1 in range(k):
            for t2 in range(k):
                sl = (slice(None), slice(t0, t0 + s * (o0 - 1) + 1, s), slice(t1, t1 + s * (o1 - 1) + 1, s),
                      slice(t2, t2 + s * (o2 - 1) + 1, s))
                dw[:, :, t0, t1, t2] = np.tensordot(dy, xp[sl], axes=([1, 2, 3], [1, 2, 3]))
                dxp[sl] += np.tensordot(w[:, :, t0, t1, t2], dy, axes=(0, 0))
    dx = dxp[:, p:p + D0, p:p + D1, p:p + D2]
    return dx, dw, dy.sum(axis=(1, 2, 3))


def batchnorm_vjp(x, gamma, mean, var, dy, eps: float = BN_EPS):
    """Gradients of the inference batch norm y = gamma (x - mean) / sigma + beta,
    sigma = sqrt(var + eps), over channel axis 0: (dx, dgamma, dbeta, dmean, dvar)."""
    g = np.asarray(gamma, np.float64)[:, None, None, None]
    mu = np.asarray(mean, np.float64)[:, None, None, None]
    v = np.asarray(var, np.float64)[:, None, None, None]
    sig = np.sqrt(v + eps)
    xc = np.asarray(x, np.float64) - mu
    ax = (1, 2, 3)
    dx = dy * g / sig
    dgamma = (dy * xc / sig).sum(axis=ax)
    dbeta = dy.sum(axis=ax)
    dmean = -(dy * g / sig).sum(axis=ax)
    dvar = (dy * g * xc * (-0.5) / (sig ** 3)).sum(axis=ax)
    return dx, dgamma, dbeta, dmean, dvar


def cnn3d_vjp(grid: np.ndarray, w, arch, dlat: np.ndarray, relu_margin: float = 0.0) -> Dict[str, np.ndarray]:
    """Gradients of the 3D-CNN latent (cf_oracle.cnn3d_forward) given dL/dlatent:
    the forward is rerun keeping every conv output before BN (c), after BN and the
    residual add (u, before the ReLU) and every activation (t); the backward walks
    the dense layers, the mean pool and the conv layers in reverse.

    relu_margin (default 0, the definition) takes each ReLU's gradient as
    [u > relu_margin]: with a small margin of either sign the result is the
    gradient a forward pass within that distance of exact arithmetic may yield,
    since pre-activations that close to 0 may fall on either side of the kink
    (a tolerance for comparing with float32 forward passes, not another model)."""
    t = [np.moveaxis(np.asarray(grid, np.float64), -1, 0)]
    cs, us = [], []
    from .cf_oracle import batchnorm, conv3d
    for i, (ci, co, k, s, r) in enumerate(arch.conv):
        c = conv3d(t[-1], w[f"conv{i}.w"], w[f"conv{i}.b"], s)
        y = batchnorm(c, w[f"bn{i}.gamma"], w[f"bn{i}.beta"], w[f"bn{i}.mean"], w[f"bn{i}.var"]) if arch.bn else c
        u = y + t[r] if r >= 0 else y
        cs.append(c)
        us.append(u)
        t.append(relu(u))
    pooled = t[-1].mean(axis=(1, 2, 3))
    dense_in, dense_pre = [], []
    lat = pooled
    names = [n for n in ("cnn_dense", "cnn_dense2") if getattr(arch, n)]
    for n in names:
        dense_in.append(lat)
        pre = _f64(w, n + ".w") @ lat + _f64(w, n + ".b")
        dense_pre.append(pre)
        lat = relu(pre)

    g: Dict[str, np.ndarray] = {}
    d = np.asarray(dlat, np.float64)
    for n, xin, pre in reversed(list(zip(names, dense_in, dense_pre))):
        dpre = d * (pre > relu_margin)
        g[n + ".w"] = np.outer(dpre, xin)
        g[n + ".b"] = dpre
        d = _f64(w, n + ".w").T @ dpre
    V = float(np.prod(t[-1].shape[1:]))
    dt = [np.zeros_like(a) for a in t]
    dt[-1] = np.broadcast_to(d[:, None, None, None] / V, t[-1].shape).copy()
    for i in reversed(range(len(arch.conv))):
        ci, co, k, s, r = arch.conv[i]
        du = dt[i + 1] * (us[i] > relu_margin)
        if r >= 0:
            dt[r] += du
        if arch.bn:
            dc, g[f"bn{i}.gamma"], g[f"bn{i}.beta"], g[f"bn{i}.mean"], g[f"bn{i}.var"] = batchnorm_vjp(
                cs[i], w[f"bn{i}.gamma"], w[f"bn{i}.mean"], w[f"bn{i}.var"], du)
        else:
            dc = du
        dx, g[f"conv{i}.w"], g[f"conv{i}.b"] = conv3d_vjp(t[i], w[f"conv{i}.w"], s, dc)
        dt[i] += dx
    return g


# --------------------------------------------------------------------------------
# SG-CNN (unstaged: embedding, K_c covalent then K_n non-covalent gated rounds,
# gated readout over ligand atoms)
# --------------------------------------------------------------------------------

def aggregate_vjp(da: np.ndarray, row_ptr: np.ndarray, col: np.ndarray) -> np.ndarray:
    """a_i = sum_{j in N(i)} h_j reversed: dh_j = sum over the rows i that list j
    of da_i (written as that scatter, not as a second aggregation)."""
    dh = np.zeros_like(da)
    for i in range(len(row_ptr) - 1):
        for e in range(int(row_ptr[i]), int(row_ptr[i + 1])):
            dh[int(col[e])] += da[i]
    return dh


def gru_cell_vjp(m, h, w_ih, w_hh, b_ih, b_hh, dh_new):
    """Gradients of h' = GRU(m, h) (gates r, z, n as cf_oracle.gru_cell) given
    dL/dh': (dm, dh, dw_ih, dw_hh, db_ih, db_hh)."""
    H = h.shape[1]
    W_ih, W_hh = np.asarray(w_ih, np.float64), np.asarray(w_hh, np.float64)
    gi = m @ W_ih.T + np.asarray(b_ih, np.float64)
    gh = h @ W_hh.T + np.asarray(b_hh, np.float64)
    r = sigmoid(gi[:, :H] + gh[:, :H])
    z = sigmoid(gi[:, H:2 * H] + gh[:, H:2 * H])
    hn = gh[:, 2 * H:]
    n = np.tanh(gi[:, 2 * H:] + r * hn)
    # h' = (1 - z) n + z h
    dn = dh_new * (1.0 - z)
    dz = dh_new * (h - n)
    dh = dh_new * z
    dpre_n = dn * (1.0 - n * n)          # n = tanh(gi_n + r * hn)
    dr = dpre_n * hn
    dhn = dpre_n * r
    dpre_z = dz * z * (1.0 - z)
    dpre_r = dr * r * (1.0 - r)
    dgi = np.concatenate([dpre_r, dpre_z, dpre_n], axis=1)
    dgh = np.concatenate([dpre_r, dpre_z, dhn], axis=1)
    dm = dgi @ W_ih
    dh = dh + dgh @ W_hh
    return dm, dh, dgi.T @ m, dgh.T @ h, dgi.sum(axis=0), dgh.sum(axis=0)


def sgcnn_vjp(feat, is_lig, cov, nc, w, arch, dsg: np.ndarray) -> Dict[str, np.ndarray]:
    """Gradients of the SG-CNN latent (cf_oracle.sgcnn_pose, unstaged) given
    dL/dlatent.  The forward is rerun keeping the state before every round and
    the round's neighbour sum and message."""
    if arch.H_nc:
        raise NotImplementedError("the staged SG-CNN has no backward here")
    x = np.asarray(feat, np.float64)
    h = x @ _f64(w, "sg.embed.w").T + _f64(w, "sg.embed.b")
    from .cf_oracle import aggregate, gru_cell
    rounds = []   # (stage, t, graph, h_in, a, m)
    for stage, K, (rp, col) in (("cov", arch.K_c, cov), ("nc", arch.K_n, nc)):
        for t in range(K):
            a = aggregate(h, rp, col)
            m = a @ _f64(w, f"sg.{stage}.msg{t}.w").T
            rounds.append((stage, t, (rp, col), h, a, m))
            h = gru_cell(m, h, w[f"sg.{stage}.gru.w_ih"], w[f"sg.{stage}.gru.w_hh"],
                         w[f"sg.{stage}.gru.b_ih"], w[f"sg.{stage}.gru.b_hh"])
    g: Dict[str, np.ndarray] = {}
    # readout s = sum_{i in lig} sigma(W_g [h_i; x_i] + b_g) * (W_v h_i + b_v)
    lig = np.asarray(is_lig).astype(bool)
    H = h.shape[1]
    hx = np.concatenate([h, x], axis=1)
    gate = sigmoid(hx @ _f64(w, "sg.gate.w").T + _f64(w, "sg.gate.b"))
    val = h @ _f64(w, "sg.val.w").T + _f64(w, "sg.val.b")
    ds = np.asarray(dsg, np.float64)
    dgate = np.where(lig[:, None], ds[None, :] * val, 0.0)
    dval = np.where(lig[:, None], ds[None, :] * gate, 0.0)
    dpre_g = dgate * gate * (1.0 - gate)
    g["sg.gate.w"] = dpre_g.T @ hx
    g["sg.gate.b"] = dpre_g.sum(axis=0)
    g["sg.val.w"] = dval.T @ h
    g["sg.val.b"] = dval.sum(axis=0)
    dh = (dpre_g @ _f64(w, "sg.gate.w"))[:, :H] + dval @ _f64(w, "sg.val.w")
    for stage in ("cov", "nc"):
        for k in ("w_ih", "w_hh", "b_ih", "b_hh"):
            g[f"sg.{stage}.gru.{k}"] = np.zeros_like(_f64(w, f"sg.{stage}.gru.{k}"))
    for stage, t, (rp, col), h_in, a, m in reversed(rounds):
        dm, dh, dwi, dwh, dbi, dbh = gru_cell_vjp(m, h_in, w[f"sg.{stage}.gru.w_ih"], w[f"sg.{stage}.gru.w_hh"],
                                                  w[f"sg.{stage}.gru.b_ih"], w[f"sg.{stage}.gru.b_hh"], dh)
        g[f"sg.{stage}.gru.w_ih"] += dwi
        g[f"sg.{stage}.gru.w_hh"] += dwh
        g[f"sg.{stage}.gru.b_ih"] += dbi
        g[f"sg.{stage}.gru.b_hh"] += dbh
        g[f"sg.{stage}.msg{t}.w"] = dm.T @ a              # m = W_t a
        dh = dh + aggregate_vjp(dm @ _f64(w, f"sg.{stage}.msg{t}.w"), rp, col)
    g["sg.embed.w"] = dh.T @ x
    g["sg.embed.b"] = dh.sum(axis=0)
    return g


# --------------------------------------------------------------------------------
# Coherent Fusion head
# --------------------------------------------------------------------------------

def selu_grad(x):
    x = np.asarray(x, np.float64)
    return np.where(x > 0, SELU_LAMBDA, SELU_LAMBDA * SELU_ALPHA * np.exp(np.minimum(x, 0.0)))


def fusion_head_vjp(cnn_lat, sg_lat, w, arch, dscore: float):
    """Gradients of the Coherent Fusion score (cf_oracle.fusion_head, coherent
    form) given dL/ds: (dcnn, dsg, grads)."""
    if arch.head != "coherent":
        raise NotImplementedError("backward covers the Coherent Fusion head")
    cnn = np.asarray(cnn_lat, np.float64)
    z = np.concatenate([cnn, np.asarray(sg_lat, np.float64)])
    layers = []   # (name, input, pre-activation)
    for l in range(arch.n_fusion - 1):
        n = "fusion.hidden" if l == 0 else f"fusion.hidden{l}"
        pre = _f64(w, n + ".w") @ z + _f64(w, n + ".b")
        layers.append((n, z, pre))
        y = selu(pre)
        z = y + z if (arch.fusion_residual and l > 0) else y
    g: Dict[str, np.ndarray] = {}
    g["fusion.out.w"] = dscore * z[None, :]
    g["fusion.out.b"] = np.array([dscore])
    dz = dscore * _f64(w, "fusion.out.w")[0]
    for l in reversed(range(len(layers))):
        n, zin, pre = layers[l]
        dpre = dz * selu_grad(pre)
        g[n + ".w"] = np.outer(dpre, zin)
        g[n + ".b"] = dpre
        dzin = _f64(w, n + ".w").T @ dpre
        dz = dzin + dz if (arch.fusion_residual and l > 0) else dzin
    nc = len(cnn)
    return dz[:nc], dz[nc:], g


# --------------------------------------------------------------------------------
# Whole path
# --------------------------------------------------------------------------------

def score_vjp(batch, w, arch, G: int, dscore, relu_margin: float = 0.0) -> Dict[str, np.ndarray]:
    """sum_p dscore[p] * d s_p / d theta for every parameter theta (zero for those
    the score does not depend on).  Grid centres are the rounded ligand centroids
    (cf_oracle.score_pose); the grid and the graphs carry no parameters.
    relu_margin: see cnn3d_vjp (0 = the definition)."""
    grads = {k: np.zeros(np.shape(v)) for k, v in w.items()}
    for p in range(batch.n_poses):
        a, b = int(batch.atom_off[p]), int(batch.atom_off[p + 1])
        xyz, feat, is_lig = batch.xyz[a:b], batch.feat[a:b], np.asarray(batch.is_lig[a:b]).astype(bool)
        center = pose_center(xyz[is_lig] if is_lig.any() else xyz)
        grid = splat_pose(xyz, feat, center, G)
        from .cf_oracle import cnn3d_forward, sgcnn_pose
        cnn_lat, _ = cnn3d_forward(grid, w, arch)
        cov = radius_graph_pose(xyz, arch.r_cov_u)
        nc = radius_graph_pose(xyz, arch.r_nc_u)
        sg_lat = sgcnn_pose(feat, is_lig, cov, nc, w, arch)
        dcnn, dsg, gh = fusion_head_vjp(cnn_lat, sg_lat, w, arch, float(dscore[p]))
        for part in (gh, cnn3d_vjp(grid, w, arch, dcnn, relu_margin), sgcnn_vjp(feat, is_lig, cov, nc, w, arch, dsg)):
            for k, v in part.items():
                grads[k] = grads[k] + np.reshape(v, grads[k].shape)
    return grads
