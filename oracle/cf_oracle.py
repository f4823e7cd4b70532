"""FP64 CPU oracle: the Coherent Fusion scoring function written out plainly.

TEST INFRASTRUCTURE ONLY (see the package docstring): the scoring library never
imports this module and shares no code with it.

The paper (Sec. 1; Sec. 2.1-2.2; Fig. 1) scores a docked pose with two heads over
two representations of the same complex -- a voxel grid read by a 3D-CNN and a
spatial graph with covalent and non-covalent edge types read by an SG-CNN
(PotentialNet on gated graph sequence networks, Sec. 3.3.1) -- whose latents are
concatenated and passed through fusion dense layers to one pK (Eq. 1; Coherent
Fusion, Sec. 3.3.3, Table V).  Featurisation, grid sizing and atom propagation are
deferred by the paper to its predecessor (Sec. 3.3), so several steps below are
readings (listed with their reasons in the design notes); each function says which.

Units: coordinates are integers in u = 2^-10 A, so every distance test is exact.
Everything else is float64.
"""
from __future__ import annotations

from typing import Dict, Optional, Sequence, Tuple

import numpy as np

U_PER_A = 1024                  # fixed-point units per Angstrom
VOXEL_U = 1024                  # grid spacing 1 A
HALF_VOXEL_U = 512
SPLAT_RCUT_U = 1536             # Gaussian truncation radius 3 sigma, sigma = 0.5 A
SPLAT_TWO_SIGMA2_U2 = 524288    # 2 sigma^2 in u^2 (sigma = 512 u)
BN_EPS = 1e-5
# SELU constants as published by Klambauer et al. (2017), the activation the paper
# selects for its fusion layers (Table V).
SELU_LAMBDA = 1.0507009873554804934193349852946
SELU_ALPHA = 1.6732632423543772848170429916717


# --------------------------------------------------------------------------------
# Grid placement and voxelisation (3D representation, Sec. 1; grid sizing and atom
# propagation deferred to the predecessor model, Sec. 3.3)
# --------------------------------------------------------------------------------

def pose_center(xyz_lig: np.ndarray) -> np.ndarray:
    """Grid centre of a pose: the ligand centroid rounded to the nearest unit,
    halves rounded up, c = floor((2*sum(x) + n) / (2*n)) per axis (integer)."""
    x = np.asarray(xyz_lig, dtype=np.int64)
    n = x.shape[0]
    s = x.sum(axis=0)
    return (2 * s + n) // (2 * n)


def voxel_center(center: np.ndarray, G: int, idx: np.ndarray) -> np.ndarray:
    """Centre of voxel idx (any integer lattice index, also outside [0, G)):
    c + (idx - (G-1)/2) * 1 A, i.e. c + 512 * (2*idx - G + 1) in u."""
    return np.asarray(center, dtype=np.int64) + HALF_VOXEL_U * (2 * np.asarray(idx, dtype=np.int64) - G + 1)


def _atom_support(X: np.ndarray, center: np.ndarray, G: int):
    """Lattice voxels (unbounded) whose centre lies within 3 sigma of atom X, with
    their squared distances in u^2."""
    c = np.asarray(center, dtype=np.int64)
    off = HALF_VOXEL_U * (G - 1)
    lo = -((-(X - c - SPLAT_RCUT_U + off)) // VOXEL_U)      # ceil
    hi = (X - c + SPLAT_RCUT_U + off) // VOXEL_U            # floor
    axes = [np.arange(lo[d], hi[d] + 1, dtype=np.int64) for d in range(3)]
    idx = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    P = voxel_center(c, G, idx)
    D = ((X[None, :] - P) ** 2).sum(axis=1)
    keep = D <= SPLAT_RCUT_U * SPLAT_RCUT_U
    return idx[keep], D[keep]


def splat_pose(xyz: np.ndarray, feat: np.ndarray, center: np.ndarray, G: int) -> np.ndarray:
    """Voxelise one pose into grid[G][G][G][C] (axes x, y, z, channel).

    Each atom spreads its feature vector over the voxels within 3 sigma of it with
    Gaussian weights w = exp(-D / (2 sigma^2)), normalised over its whole
    (unclipped) support so every atom carries unit mass; the normaliser is summed
    in ascending-distance order.  Voxels outside the grid are dropped.  Atoms are
    added in index order.
    """
    xyz = np.asarray(xyz, dtype=np.int64)
    feat = np.asarray(feat, dtype=np.float64)
    grid = np.zeros((G, G, G, feat.shape[1]), dtype=np.float64)
    for a in range(xyz.shape[0]):
        idx, D = _atom_support(xyz[a], center, G)
        w = np.exp(-D.astype(np.float64) / SPLAT_TWO_SIGMA2_U2)
        Z = 0.0
        for v in w[np.argsort(D, kind="stable")]:
            Z += v
        inside = np.all((idx >= 0) & (idx < G), axis=1)
        for (i, j, k), wv in zip(idx[inside], w[inside]):
            grid[i, j, k, :] += feat[a] * (wv / Z)
    return grid


def splat_batch(batch, centers: np.ndarray, G: int) -> np.ndarray:
    P = batch.n_poses
    out = np.zeros((P, G, G, G, batch.feat.shape[1]))
    for p in range(P):
        a, b = int(batch.atom_off[p]), int(batch.atom_off[p + 1])
        out[p] = splat_pose(batch.xyz[a:b], batch.feat[a:b], centers[p], G)
    return out


# --------------------------------------------------------------------------------
# 3D-CNN (Sec. 3.3.1, Table III: conv filters, residual connection, dense nodes)
# --------------------------------------------------------------------------------

def conv3d(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int) -> np.ndarray:
    """Cross-correlation with zero 'same' padding p = (k-1)/2:
    out[o, i0, i1, i2] = b[o] + sum_{c, t0, t1, t2} w[o, c, t0, t1, t2] *
                         x[c, s*i0 + t0 - p, s*i1 + t1 - p, s*i2 + t2 - p].
    The sum over c for one tap (t0, t1, t2) is a matrix product; taps are
    accumulated one after another.  x: [C, D0, D1, D2]; w: [O, C, k, k, k]."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    C, D0, D1, D2 = x.shape
    O, C2, k = w.shape[0], w.shape[1], w.shape[2]
    assert C2 == C
    p = (k - 1) // 2
    s = stride
    o0, o1, o2 = [(d + 2 * p - k) // s + 1 for d in (D0, D1, D2)]
    xp = np.zeros((C, D0 + 2 * p, D1 + 2 * p, D2 + 2 * p))
    xp[:, p:p + D0, p:p + D1, p:p + D2] = x
    out = np.empty((O, o0, o1, o2))
    out[:] = np.asarray(b, dtype=np.float64)[:, None, None, None]
    for t0 in range(k):
        for t1 in range(k):
            for t2 in range(k):
                patch = xp[:, t0:t0 + s * (o0 - 1) + 1:s, t1:t1 + s * (o1 - 1) + 1:s,
                           t2:t2 + s * (o2 - 1) + 1:s]
                out += np.tensordot(w[:, :, t0, t1, t2], patch, axes=(1, 0))
    return out


def batchnorm(x: np.ndarray, gamma, beta, mean, var, eps: float = BN_EPS) -> np.ndarray:
    """Inference batch norm over the channel axis 0."""
    g = np.asarray(gamma, np.float64)[:, None, None, None]
    bt = np.asarray(beta, np.float64)[:, None, None, None]
    mu = np.asarray(mean, np.float64)[:, None, None, None]
    v = np.asarray(var, np.float64)[:, None, None, None]
    return g * (x - mu) / np.sqrt(v + eps) + bt


def relu(x):
    return np.maximum(x, 0.0)


def cnn3d_forward(grid: np.ndarray, w: Dict[str, np.ndarray], arch) -> Tuple[np.ndarray, list]:
    """grid [G,G,G,C] -> (latent, per-layer activations).  Each conv is followed by
    BN (if enabled) and ReLU; a residual conv adds its block input before the
    ReLU; global average pooling; up to two dense + ReLU layers."""
    t = [np.moveaxis(np.asarray(grid, np.float64), -1, 0)]
    for i, (ci, co, k, s, r) in enumerate(arch.conv):
        y = conv3d(t[-1], w[f"conv{i}.w"], w[f"conv{i}.b"], s)
        if arch.bn:
            y = batchnorm(y, w[f"bn{i}.gamma"], w[f"bn{i}.beta"], w[f"bn{i}.mean"], w[f"bn{i}.var"])
        if r >= 0:
            y = y + t[r]
        t.append(relu(y))
    pooled = t[-1].mean(axis=(1, 2, 3))
    lat = pooled
    for name in ("cnn_dense", "cnn_dense2"):
        if getattr(arch, name):
            lat = relu(np.asarray(w[name + ".w"], np.float64) @ lat + np.asarray(w[name + ".b"], np.float64))
    return lat, t


# --------------------------------------------------------------------------------
# Spatial graph (Sec. 1: edge types by distance threshold; Table I / II thresholds)
# --------------------------------------------------------------------------------

def radius_graph_pose(xyz: np.ndarray, r_u: int) -> Tuple[np.ndarray, np.ndarray]:
    """All ordered pairs (i, j), i != j, with |x_i - x_j|^2 <= r^2 (exact integers).
    Returns CSR (row_ptr [n+1], col) with rows by atom and columns ascending."""
    X = np.asarray(xyz, dtype=np.int64)
    d = X[:, None, :] - X[None, :, :]
    D = (d * d).sum(axis=-1)
    A = D <= np.int64(r_u) * np.int64(r_u)
    np.fill_diagonal(A, False)
    _, cols = np.nonzero(A)
    row_ptr = np.zeros(X.shape[0] + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(A.sum(axis=1))
    return row_ptr, cols.astype(np.int64)


def radius_graph_batch(batch, r_u: int) -> Tuple[np.ndarray, np.ndarray]:
    """Per-pose graphs concatenated with global atom ids (edges never cross poses)."""
    rps, cols = [np.zeros(1, dtype=np.int64)], []
    base_e = 0
    for p in range(batch.n_poses):
        a, b = int(batch.atom_off[p]), int(batch.atom_off[p + 1])
        rp, c = radius_graph_pose(batch.xyz[a:b], r_u)
        rps.append(rp[1:] + base_e)
        cols.append(c + a)
        base_e += int(rp[-1])
    return np.concatenate(rps), (np.concatenate(cols) if cols else np.zeros(0, np.int64))


# --------------------------------------------------------------------------------
# SG-CNN (PotentialNet on gated graph sequence networks, Sec. 3.3.1, Table II)
# --------------------------------------------------------------------------------

def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def gru_cell(m: np.ndarray, h: np.ndarray, w_ih, w_hh, b_ih, b_hh) -> np.ndarray:
    """Gated recurrent unit update h' = GRU(m, h) with gates stacked (r, z, n):
    r = s(W_ir m + b_ir + W_hr h + b_hr), z = s(W_iz m + b_iz + W_hz h + b_hz),
    n = tanh(W_in m + b_in + r * (W_hn h + b_hn)), h' = (1 - z) * n + z * h."""
    H = h.shape[1]
    gi = m @ np.asarray(w_ih, np.float64).T + np.asarray(b_ih, np.float64)
    gh = h @ np.asarray(w_hh, np.float64).T + np.asarray(b_hh, np.float64)
    r = sigmoid(gi[:, :H] + gh[:, :H])
    z = sigmoid(gi[:, H:2 * H] + gh[:, H:2 * H])
    n = np.tanh(gi[:, 2 * H:] + r * gh[:, 2 * H:])
    return (1.0 - z) * n + z * h


def aggregate(h: np.ndarray, row_ptr: np.ndarray, col: np.ndarray) -> np.ndarray:
    """a_i = sum of h_j over the neighbours j of i (unweighted, no self term)."""
    a = np.zeros_like(h)
    for i in range(h.shape[0]):
        js = col[row_ptr[i]:row_ptr[i + 1]]
        if len(js):
            a[i] = h[js].sum(axis=0)
    return a


def sgcnn_pose(feat: np.ndarray, is_lig: np.ndarray, cov, nc, w: Dict[str, np.ndarray], arch,
               return_h: bool = False):
    """One pose: embed, K_c covalent rounds then K_n non-covalent rounds of
    a = sum of neighbour states, m = W_t a, h <- GRU_stage(m, h), then the gated
    readout over ligand atoms s = sum_i sigma(W_g [h_i; u_i] + b_g) * (W_v h_i + b_v),
    where u is the stage input (the raw features x).

    With PotentialNet staging (arch.H_nc > 0, Sec. 3.3.1 / Table II gather widths),
    the covalent stage closes with a per-atom gated gather
    g_i = sigma(W_g1 [h_i; x_i] + b_g1) * (W_v1 h_i + b_v1) (width H); the
    non-covalent stage starts from a linear embedding of g (width H_nc), and the
    final readout's gate reads [h_i; g_i].  cov / nc are local CSR pairs."""
    x = np.asarray(feat, np.float64)
    f64 = lambda k: np.asarray(w[k], np.float64)
    h = x @ f64("sg.embed.w").T + f64("sg.embed.b")
    u = x
    for stage, K, (rp, col) in (("cov", arch.K_c, cov), ("nc", arch.K_n, nc)):
        if stage == "nc" and arch.H_nc:
            g = sigmoid(np.concatenate([h, x], axis=1) @ f64("sg.mid.gate.w").T + f64("sg.mid.gate.b")) \
                * (h @ f64("sg.mid.val.w").T + f64("sg.mid.val.b"))
            h = g @ f64("sg.embed2.w").T + f64("sg.embed2.b")
            u = g
        for t in range(K):
            a = aggregate(h, rp, col)
            m = a @ f64(f"sg.{stage}.msg{t}.w").T
            h = gru_cell(m, h, w[f"sg.{stage}.gru.w_ih"], w[f"sg.{stage}.gru.w_hh"],
                         w[f"sg.{stage}.gru.b_ih"], w[f"sg.{stage}.gru.b_hh"])
    gate = sigmoid(np.concatenate([h, u], axis=1) @ f64("sg.gate.w").T + f64("sg.gate.b"))
    val = h @ f64("sg.val.w").T + f64("sg.val.b")
    lig = np.asarray(is_lig).astype(bool)
    s = (gate[lig] * val[lig]).sum(axis=0)
    return (s, h) if return_h else s


def sgcnn_batch(batch, w, arch) -> np.ndarray:
    out = np.zeros((batch.n_poses, arch.sg_latent))
    for p in range(batch.n_poses):
        a, b = int(batch.atom_off[p]), int(batch.atom_off[p + 1])
        cov = radius_graph_pose(batch.xyz[a:b], arch.r_cov_u)
        nc = radius_graph_pose(batch.xyz[a:b], arch.r_nc_u)
        out[p] = sgcnn_pose(batch.feat[a:b], batch.is_lig[a:b], cov, nc, w, arch)
    return out


# --------------------------------------------------------------------------------
# Fusion heads (Coherent Fusion, Sec. 2.2, Table V; Mid-level and Late Fusion,
# Sec. 2.1, Table IV)
# --------------------------------------------------------------------------------

def selu(x):
    x = np.asarray(x, np.float64)
    return np.where(x > 0, SELU_LAMBDA * x, SELU_LAMBDA * SELU_ALPHA * np.expm1(np.minimum(x, 0.0)))


def _dense(w, name, x):
    return np.asarray(w[name + ".w"], np.float64) @ x + np.asarray(w[name + ".b"], np.float64)


def fusion_block(z: np.ndarray, w, arch) -> float:
    """The fusion dense layers (Fig. 1, fusion block; Tables IV-V): n_fusion - 1
    hidden SELU layers of width fusion_hidden -- with residual fusion layers, each
    hidden layer after the first adds its own input to its output -- then a linear
    layer to one pK.  Dropout is the identity at inference."""
    for l in range(arch.n_fusion - 1):
        y = selu(_dense(w, "fusion.hidden" if l == 0 else f"fusion.hidden{l}", z))
        z = y + z if (arch.fusion_residual and l > 0) else y
    return float(_dense(w, "fusion.out", z)[0])


def fusion_head(cnn_lat: np.ndarray, sg_lat: np.ndarray, w, arch) -> float:
    """pK of one pose from its two latents, per the model's fusion form.

    coherent (Sec. 2.2, Table V): fusion block over [cnn; sg].
    mid (Mid-level Fusion, Sec. 2.1, Table IV): each latent first passes through
        its own model-specific SELU dense layer (same width); those outputs are
        concatenated with the raw latents, [u_cnn; u_sg; cnn; sg], and fed to the
        fusion block.
    late (Late Fusion, Sec. 2.1): each branch predicts a pK on its own -- the
        3D-CNN by a linear layer on its latent, the SG-CNN by its ReLU dense layers
        and a linear layer -- and the score is the unweighted mean of the two.
    """
    cnn = np.asarray(cnn_lat, np.float64)
    sg = np.asarray(sg_lat, np.float64)
    if arch.head == "late":
        pk_cnn = _dense(w, "late.cnn_out", cnn)[0]
        x = sg
        for j in range(len(arch.sg_dense)):
            x = np.maximum(_dense(w, f"late.sg_dense{j}", x), 0.0)
        pk_sg = _dense(w, "late.sg_out", x)[0]
        return float(late_fusion(pk_cnn, pk_sg))
    if arch.head == "mid":
        z = np.concatenate([selu(_dense(w, "mid.cnn", cnn)), selu(_dense(w, "mid.sg", sg)), cnn, sg])
    else:
        z = np.concatenate([cnn, sg])
    return fusion_block(z, w, arch)


def late_fusion(pk_cnn, pk_sg):
    """Late Fusion (Sec. 2.1): unweighted arithmetic mean of the two heads' pK."""
    return (np.asarray(pk_cnn, np.float64) + np.asarray(pk_sg, np.float64)) / 2.0


# --------------------------------------------------------------------------------
# Whole path
# --------------------------------------------------------------------------------

def score_pose(xyz, feat, is_lig, w, arch, G: int, center: Optional[np.ndarray] = None,
               detail: bool = False):
    is_lig = np.asarray(is_lig).astype(bool)
    if center is None:   # grid centre: ligand centroid, or all atoms' if the pose has no ligand atom
        center = pose_center(np.asarray(xyz)[is_lig] if is_lig.any() else np.asarray(xyz))
    grid = splat_pose(xyz, feat, center, G)
    cnn_lat, _ = cnn3d_forward(grid, w, arch)
    cov = radius_graph_pose(xyz, arch.r_cov_u)
    nc = radius_graph_pose(xyz, arch.r_nc_u)
    sg_lat = sgcnn_pose(feat, is_lig, cov, nc, w, arch)
    s = fusion_head(cnn_lat, sg_lat, w, arch)
    if detail:
        return s, dict(center=center, grid=grid, cnn_lat=cnn_lat, sg_lat=sg_lat, cov=cov, nc=nc)
    return s


def score_batch(batch, w, arch, G: int, poses: Optional[Sequence[int]] = None,
                workers: int = 1) -> np.ndarray:
    """Scores of the given poses (all by default).  workers > 1 scores poses in
    separate processes (each pose is independent)."""
    poses = list(range(batch.n_poses)) if poses is None else list(poses)
    args = []
    for p in poses:
        a, b = int(batch.atom_off[p]), int(batch.atom_off[p + 1])
        args.append((batch.xyz[a:b], batch.feat[a:b], batch.is_lig[a:b]))
    if workers <= 1:
        return np.array([score_pose(x, f, l, w, arch, G) for (x, f, l) in args])
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        res = pool.starmap(_score_one, [(x, f, l, w, arch, G) for (x, f, l) in args])
    return np.array(res)


def _score_one(x, f, l, w, arch, G):
    return score_pose(x, f, l, w, arch, G)


# --------------------------------------------------------------------------------
# Selection after scoring (Sec. 5.2: a compound is represented by its strongest
# prediction over all its docked poses -- the maximum Fusion pK; Sec. 3.4: the best
# 100 of a million screened compounds are bought)
# --------------------------------------------------------------------------------

def compound_best(scores, compound_off):
    """Per segment [off[c], off[c+1]): (max score, lowest index attaining it);
    NaN scores are ignored; an empty or all-NaN segment gives (-inf, -1)."""
    best, idx = [], []
    for c in range(len(compound_off) - 1):
        b, i = -np.inf, -1
        for p in range(int(compound_off[c]), int(compound_off[c + 1])):
            v = float(scores[p])
            if v == v and (i < 0 or v > b):
                b, i = v, p
        best.append(b)
        idx.append(i)
    return np.array(best), np.array(idx, dtype=np.int64)


def top_k(values, k: int):
    """Indices of the k largest values in descending order; equal values by lower
    index; NaN after every number."""
    v = np.asarray(values, dtype=np.float64)
    keyed = sorted(range(len(v)), key=lambda i: (1, 0.0, i) if v[i] != v[i] else (0, -v[i], i))
    return np.array(keyed[:k], dtype=np.int64)
