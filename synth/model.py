"""Model architectures, workload configurations and seeded random weights.

Architectures follow the paper's structure (Sec. 2.2, Fig. 1, Sec. 3.3): a 3D-CNN
over a voxel grid and a PotentialNet/GGNN-style SG-CNN over a two-edge-type
spatial graph, whose latents are concatenated into fusion dense layers ending in
one pK (Eq. 1).  Layer sizes are those of the two workloads this project measures
(a tiny model and a full-size model); the paper's own tuned sizes (Tables II-V)
are a different workload.

Weight draws (a reading; the paper trains its weights and ships none):
  W ~ N(0, 2/fan_in) (He-normal), biases ~ N(0, 0.01^2),
  BatchNorm gamma ~ U[0.8, 1.2], beta, running mean ~ N(0, 0.05^2),
  running var ~ U[0.8, 1.2].
Every tensor has its own SplitMix64 counter stream keyed by (seed, tensor index),
in the fixed order of `param_shapes`.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Tuple

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * M1
    z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def _stream(key: int, n: int) -> np.ndarray:
    """First n SplitMix64 outputs from state `key` (counter form)."""
    with np.errstate(over="ignore"):
        i = np.arange(1, n + 1, dtype=np.uint64)
        return _mix64(np.uint64(key) + i * GOLDEN)


def _key(seed: int, tag: int) -> int:
    with np.errstate(over="ignore"):
        k = _mix64(np.array([seed], dtype=np.uint64) * GOLDEN + np.uint64(tag))
    return int(k[0])


def _uniform(key: int, n: int) -> np.ndarray:
    return (_stream(key, n) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def _normal(key: int, n: int) -> np.ndarray:
    u = _uniform(key, 2 * n)
    u1 = np.maximum(u[0::2], 1e-300)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u[1::2])


@dataclasses.dataclass(frozen=True)
class ModelArch:
    """Structure of one Coherent Fusion model.

    conv: tuples (c_in, c_out, k, stride, res_src).  Tensor t0 is the voxel grid and
    t_{i+1} the output of conv i; res_src >= 0 adds tensor t_{res_src} before the
    ReLU of conv i (the second conv of a residual block adds the block input).
    """
    name: str
    n_ch: int
    conv: Tuple[Tuple[int, int, int, int, int], ...]
    bn: bool
    cnn_dense: int          # 0: latent = pooled features; else dense + ReLU to this width
    H: int                  # SG-CNN hidden width (= gather width)
    K_c: int                # covalent propagation rounds
    K_n: int                # non-covalent propagation rounds
    r_cov_u: int            # covalent cutoff, units of 2^-10 A
    r_nc_u: int             # non-covalent cutoff, units of 2^-10 A
    fusion_hidden: int      # width of the fusion block's hidden SELU layers (0: none)
    fusion_layers: int = 0  # dense layers of the fusion block incl. the output layer
                            # (0: one hidden layer if fusion_hidden, else linear)
    fusion_residual: bool = False   # hidden layers after the first add their input
    head: str = "coherent"  # "coherent" / "mid": fusion block over the latents
                            # ("mid" first passes each latent through its own SELU
                            # dense layer and concatenates those with the raw
                            # latents); "late": each branch predicts its own pK
                            # and the score is their mean
    sg_dense: Tuple[int, ...] = ()  # late head: SG-CNN dense layers (ReLU) before its output
    cnn_dense2: int = 0     # second 3D-CNN dense layer (ReLU) after cnn_dense, 0 = none
    H_nc: int = 0           # > 0: PotentialNet staging -- the covalent stage runs at width H,
                            # a per-atom gated gather closes it, and the non-covalent stage
                            # runs at width H_nc on a linear embedding of that gather

    @property
    def n_fusion(self) -> int:
        return self.fusion_layers if self.fusion_layers else (2 if self.fusion_hidden else 1)

    @property
    def head_outputs(self) -> Tuple[str, ...]:
        """Parameter prefixes of the layers that produce a pK (calibrated)."""
        return ("late.cnn_out", "late.sg_out") if self.head == "late" else ("fusion.out",)

    @property
    def c_last(self) -> int:
        return self.conv[-1][1]

    @property
    def cnn_latent(self) -> int:
        return self.cnn_dense2 or self.cnn_dense or self.c_last

    @property
    def sg_latent(self) -> int:
        return self.H_nc or self.H

    @property
    def fusion_in(self) -> int:
        return (2 if self.head == "mid" else 1) * (self.cnn_latent + self.sg_latent)

    def out_dims(self, G: int) -> List[int]:
        dims = [G]
        for (_, _, k, s, _) in self.conv:
            p = (k - 1) // 2
            dims.append((dims[-1] + 2 * p - k) // s + 1)
        return dims

    def flops_per_pose(self, G: int) -> float:
        """Multiply-add FLOPs of the conv stack (2 per MAC), the dominant term."""
        dims = self.out_dims(G)
        f = 0.0
        for i, (ci, co, k, s, _) in enumerate(self.conv):
            f += 2.0 * ci * co * k ** 3 * dims[i + 1] ** 3
        return f


R_COV_U = int(round(1.6 * 1024))   # 1638
R_NC_U = int(round(4.5 * 1024))    # 4608
R_COV_PAPER_U = int(round(2.24 * 1024))   # 2294 (Table II)
R_NC_PAPER_U = int(round(5.22 * 1024))    # 5345 (Table II)

ARCHS: Dict[str, ModelArch] = {
    "tiny": ModelArch("tiny", 19, ((19, 16, 5, 1, -1), (16, 16, 5, 1, -1)), True, 0,
                      16, 1, 1, R_COV_U, R_NC_U, 0),
    "full": ModelArch("full", 19,
                      ((19, 64, 7, 2, -1), (64, 64, 7, 1, -1), (64, 64, 7, 1, 1),
                       (64, 64, 7, 1, -1), (64, 64, 7, 1, 3), (64, 128, 7, 2, -1)),
                      True, 10, 64, 3, 3, R_COV_U, R_NC_U, 64),
}
# The same trunk (identical conv / SG-CNN weights: head parameters are drawn
# last) under the two earlier fusion forms the paper compares against (Sec. 2.1,
# Sec. 3.3.2, Table IV): Mid-level Fusion with model-specific layers and five
# residual fusion layers, and Late Fusion with the SG-CNN's own dense layers
# (gather width reduced by 1.5, then by 2).
ARCHS["full_mid"] = dataclasses.replace(ARCHS["full"], name="full_mid", head="mid", fusion_layers=5,
                                        fusion_residual=True)
ARCHS["full_late"] = dataclasses.replace(ARCHS["full"], name="full_late", head="late", fusion_hidden=0,
                                         sg_dense=(42, 21))

# The paper's own tuned sizes as a second workload (Sec. 3.3.1, Tables II, III, V):
# 3D-CNN with 32 filters of 5^3 then 64 of 3^3, residual connections around the
# stride-1 pairs, no BatchNorm, dense layers of 128 and 128 / 2 nodes; SG-CNN with
# 6 covalent rounds at gather width 24 and 3 non-covalent rounds at width 128,
# cutoffs 2.24 / 5.22 A; Coherent Fusion head of 4 fusion layers.
ARCHS["paper"] = ModelArch("paper", 19,
                           ((19, 32, 5, 2, -1), (32, 32, 5, 1, -1), (32, 32, 5, 1, 1),
                            (32, 64, 3, 2, -1), (64, 64, 3, 1, -1), (64, 64, 3, 1, 4)),
                           False, 128, 24, 6, 3, R_COV_PAPER_U, R_NC_PAPER_U, 64,
                           fusion_layers=4, cnn_dense2=64, H_nc=128)

# Workloads.  mode 0: n_lig ~ U{lim0..lim1}, n_pocket ~ U{lim2..lim3};
# mode 1: total ~ log-U[lim0, lim1] split into ligand / pocket.
CONFIGS = {
    "c1": dict(arch="tiny", G=24, n_poses=64, stream=1, mode=0, lim=(20, 40, 150, 300)),
    "c2": dict(arch="full", G=48, n_poses=4096, stream=2, mode=0, lim=(20, 60, 400, 900)),
    "c4": dict(arch="full", G=(32, 48, 64), n_poses=32768, stream=4, mode=1, lim=(200, 1500)),
    "c5": dict(arch="full", G=(48, 64), n_poses=1_000_000, stream=5, mode=1, lim=(200, 1500)),
}


def param_shapes(arch: ModelArch) -> List[Tuple[str, Tuple[int, ...], str]]:
    """(name, shape, init kind) in the fixed draw order."""
    out: List[Tuple[str, Tuple[int, ...], str]] = []
    for i, (ci, co, k, s, r) in enumerate(arch.conv):
        out.append((f"conv{i}.w", (co, ci, k, k, k), "he"))
        out.append((f"conv{i}.b", (co,), "bias"))
        if arch.bn:
            out.append((f"bn{i}.gamma", (co,), "gamma"))
            out.append((f"bn{i}.beta", (co,), "beta"))
            out.append((f"bn{i}.mean", (co,), "beta"))
            out.append((f"bn{i}.var", (co,), "var"))
    if arch.cnn_dense:
        out.append(("cnn_dense.w", (arch.cnn_dense, arch.c_last), "he"))
        out.append(("cnn_dense.b", (arch.cnn_dense,), "bias"))
    if arch.cnn_dense2:
        out.append(("cnn_dense2.w", (arch.cnn_dense2, arch.cnn_dense), "he"))
        out.append(("cnn_dense2.b", (arch.cnn_dense2,), "bias"))
    H = arch.H
    out.append(("sg.embed.w", (H, arch.n_ch), "he"))
    out.append(("sg.embed.b", (H,), "bias"))
    for stage, K in (("cov", arch.K_c), ("nc", arch.K_n)):
        if stage == "nc" and arch.H_nc:
            out.append(("sg.mid.gate.w", (H, H + arch.n_ch), "he"))
            out.append(("sg.mid.gate.b", (H,), "bias"))
            out.append(("sg.mid.val.w", (H, H), "he"))
            out.append(("sg.mid.val.b", (H,), "bias"))
            out.append(("sg.embed2.w", (arch.H_nc, H), "he"))
            out.append(("sg.embed2.b", (arch.H_nc,), "bias"))
            H = arch.H_nc
        for t in range(K):
            out.append((f"sg.{stage}.msg{t}.w", (H, H), "he"))
        out.append((f"sg.{stage}.gru.w_ih", (3 * H, H), "he"))
        out.append((f"sg.{stage}.gru.w_hh", (3 * H, H), "he"))
        out.append((f"sg.{stage}.gru.b_ih", (3 * H,), "bias"))
        out.append((f"sg.{stage}.gru.b_hh", (3 * H,), "bias"))
    # the final gate reads [h; stage input]: the raw features, or the covalent gather
    out.append(("sg.gate.w", (H, H + (arch.H if arch.H_nc else arch.n_ch)), "he"))
    out.append(("sg.gate.b", (H,), "bias"))
    out.append(("sg.val.w", (H, H), "he"))
    out.append(("sg.val.b", (H,), "bias"))
    lc = arch.cnn_latent
    if arch.head == "late":
        out.append(("late.cnn_out.w", (1, lc), "he"))
        out.append(("late.cnn_out.b", (1,), "bias"))
        prev = arch.sg_latent
        for j, d in enumerate(arch.sg_dense):
            out.append((f"late.sg_dense{j}.w", (d, prev), "he"))
            out.append((f"late.sg_dense{j}.b", (d,), "bias"))
            prev = d
        out.append(("late.sg_out.w", (1, prev), "he"))
        out.append(("late.sg_out.b", (1,), "bias"))
        return out
    if arch.head == "mid":
        Hs = arch.sg_latent
        out.append(("mid.cnn.w", (lc, lc), "he"))
        out.append(("mid.cnn.b", (lc,), "bias"))
        out.append(("mid.sg.w", (Hs, Hs), "he"))
        out.append(("mid.sg.b", (Hs,), "bias"))
    prev = arch.fusion_in
    for l in range(arch.n_fusion - 1):
        name = "fusion.hidden" if l == 0 else f"fusion.hidden{l}"
        out.append((f"{name}.w", (arch.fusion_hidden, prev), "he"))
        out.append((f"{name}.b", (arch.fusion_hidden,), "bias"))
        prev = arch.fusion_hidden
    out.append(("fusion.out.w", (1, prev), "he"))
    out.append(("fusion.out.b", (1,), "bias"))
    return out


def n_params(arch: ModelArch) -> int:
    return int(sum(np.prod(s) for _, s, _ in param_shapes(arch)))


def make_weights(arch: ModelArch, seed: int = 1) -> Dict[str, np.ndarray]:
    """Seeded random weights (float32), keyed by parameter name."""
    w: Dict[str, np.ndarray] = {}
    for idx, (name, shape, kind) in enumerate(param_shapes(arch)):
        n = int(np.prod(shape))
        key = _key(seed, 0x5EED0000 + idx)
        if kind == "he":
            fan_in = int(np.prod(shape[1:]))
            v = _normal(key, n) * np.sqrt(2.0 / fan_in)
        elif kind == "bias":
            v = _normal(key, n) * 0.01
        elif kind == "beta":
            v = _normal(key, n) * 0.05
        elif kind in ("gamma", "var"):
            v = 0.8 + 0.4 * _uniform(key, n)
        else:
            raise ValueError(kind)
        w[name] = v.astype(np.float32).reshape(shape)
    return w


def apply_calibration(w: Dict[str, np.ndarray], scale: float, shift: float) -> Dict[str, np.ndarray]:
    """Affine rescale of the output layer: score' = scale * score + shift.

    Random weights give scores on an arbitrary scale, which would make an error
    bound in pK units meaningless; the calibration (scale, shift) that maps a
    config's first 64 oracle scores to mean 6.0 / std 1.5 pK is stored beside the
    test fixtures and applied here to the last layer only.
    """
    out = dict(w)
    for o in _outputs_of(w):   # Late Fusion: both branch outputs, so their mean maps the same way
        out[o + ".w"] = (w[o + ".w"].astype(np.float64) * scale).astype(np.float32)
        out[o + ".b"] = (w[o + ".b"].astype(np.float64) * scale + shift).astype(np.float32)
    return out


def _outputs_of(w: Dict[str, np.ndarray]) -> Tuple[str, ...]:
    return ("late.cnn_out", "late.sg_out") if "late.cnn_out.w" in w else ("fusion.out",)
