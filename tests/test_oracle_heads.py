"""Pins of the oracle's fusion heads (Coherent, Mid-level and Late Fusion) that do
not re-type its formulas: structural reductions (zeroed layers that must vanish or
pass their input through), closed forms, a torch float64 composition of library
layers, and the calibration's affine action."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
import synth


def _latents(arch, seed=0):
    rng = np.random.default_rng(seed)
    return np.abs(rng.normal(size=arch.cnn_latent)), rng.normal(size=arch.H)


def _torch_head(arch, w, cnn, sg):
    """The same heads assembled from torch.nn layers in float64."""
    def lin(name):
        W = torch.from_numpy(w[name + ".w"].astype(np.float64))
        m = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            m.weight.copy_(W)
            m.bias.copy_(torch.from_numpy(w[name + ".b"].astype(np.float64)))
        return m

    c = torch.from_numpy(cnn)
    s = torch.from_numpy(sg)
    with torch.no_grad():
        if arch.head == "late":
            layers = []
            for j in range(len(arch.sg_dense)):
                layers += [lin(f"late.sg_dense{j}"), torch.nn.ReLU()]
            sg_branch = torch.nn.Sequential(*layers, lin("late.sg_out"))
            return float(((lin("late.cnn_out")(c) + sg_branch(s)) / 2)[0])
        if arch.head == "mid":
            z = torch.cat([torch.nn.SELU()(lin("mid.cnn")(c)), torch.nn.SELU()(lin("mid.sg")(s)), c, s])
        else:
            z = torch.cat([c, s])
        for l in range(arch.n_fusion - 1):
            y = torch.nn.SELU()(lin("fusion.hidden" if l == 0 else f"fusion.hidden{l}")(z))
            z = y + z if (arch.fusion_residual and l > 0) else y
        return float(lin("fusion.out")(z)[0])


@pytest.mark.parametrize("name", ["tiny", "full", "full_mid", "full_late"])
def test_head_matches_torch_layers(name):
    arch = synth.ARCHS[name]
    w = synth.make_weights(arch)
    for seed in range(3):
        cnn, sg = _latents(arch, seed)
        ref = _torch_head(arch, w, cnn, sg)
        assert oracle.fusion_head(cnn, sg, w, arch) == pytest.approx(ref, rel=1e-12, abs=1e-12)


def test_mid_with_silent_specific_layers_is_coherent_on_the_raw_columns():
    # zero model-specific layers output SELU(0) = 0, so only the raw-latent columns
    # of the first fusion layer act: a wrong concatenation order fails here
    arch = synth.ARCHS["full_mid"]
    w = dict(synth.make_weights(arch))
    for k in ("mid.cnn.w", "mid.cnn.b", "mid.sg.w", "mid.sg.b"):
        w[k] = np.zeros_like(w[k])
    n_raw = arch.cnn_latent + arch.H
    coh = dataclasses.replace(arch, head="coherent")
    wc = dict(w)
    wc["fusion.hidden.w"] = w["fusion.hidden.w"][:, n_raw:]
    cnn, sg = _latents(arch, 5)
    assert oracle.fusion_head(cnn, sg, w, arch) == pytest.approx(oracle.fusion_head(cnn, sg, wc, coh), rel=1e-13)


def test_zeroed_residual_layers_pass_their_input_through():
    # a residual hidden layer with zero weights and bias adds SELU(0) = 0: the
    # network equals the one without those layers (without the skip it would
    # collapse to the output bias)
    arch = synth.ARCHS["full_mid"]
    w = dict(synth.make_weights(arch))
    for l in range(1, arch.n_fusion - 1):
        w[f"fusion.hidden{l}.w"] = np.zeros_like(w[f"fusion.hidden{l}.w"])
        w[f"fusion.hidden{l}.b"] = np.zeros_like(w[f"fusion.hidden{l}.b"])
    short = dataclasses.replace(arch, fusion_layers=2)
    cnn, sg = _latents(arch, 6)
    got = oracle.fusion_head(cnn, sg, w, arch)
    assert got == pytest.approx(oracle.fusion_head(cnn, sg, w, short), rel=1e-13)
    assert abs(got - float(w["fusion.out.b"][0])) > 1e-3


def test_late_fusion_closed_form():
    # SG dense layers that select leading coordinates of a non-negative latent
    # (ReLU is then the identity), so the score is a hand-computable mean
    arch = synth.ARCHS["full_late"]
    d0, d1 = arch.sg_dense
    w = dict(synth.make_weights(arch))
    w["late.sg_dense0.w"] = np.eye(d0, arch.H, dtype=np.float32)
    w["late.sg_dense0.b"] = np.zeros(d0, np.float32)
    w["late.sg_dense1.w"] = np.eye(d1, d0, dtype=np.float32)
    w["late.sg_dense1.b"] = np.zeros(d1, np.float32)
    rng = np.random.default_rng(9)
    cnn = rng.normal(size=arch.cnn_latent)
    sg = np.abs(rng.normal(size=arch.H))
    wc, bc = w["late.cnn_out.w"][0].astype(np.float64), float(w["late.cnn_out.b"][0])
    ws, bs = w["late.sg_out.w"][0].astype(np.float64), float(w["late.sg_out.b"][0])
    pk_cnn = sum(wc[i] * cnn[i] for i in range(arch.cnn_latent)) + bc
    pk_sg = sum(ws[i] * sg[i] for i in range(d1)) + bs
    assert oracle.fusion_head(cnn, sg, w, arch) == pytest.approx(0.5 * (pk_cnn + pk_sg), rel=1e-13)
    # negative entries beyond the selected ones must not matter; negative selected ones are clipped
    sg2 = sg.copy()
    sg2[d1:] = -5.0
    sg2[0] = -1.0
    pk_sg2 = sum(ws[i] * max(sg2[i], 0.0) for i in range(d1)) + bs
    assert oracle.fusion_head(cnn, sg2, w, arch) == pytest.approx(0.5 * (pk_cnn + pk_sg2), rel=1e-13)


@pytest.mark.parametrize("name", ["full", "full_mid", "full_late"])
def test_calibration_is_affine_on_the_score(name):
    arch = synth.ARCHS[name]
    w = synth.make_weights(arch)
    cw = synth.apply_calibration(w, 0.37, 4.25)
    for seed in range(3):
        cnn, sg = _latents(arch, seed)
        raw = oracle.fusion_head(cnn, sg, w, arch)
        assert oracle.fusion_head(cnn, sg, cw, arch) == pytest.approx(0.37 * raw + 4.25, rel=1e-6, abs=1e-6)


def test_head_variants_share_the_trunk():
    full = synth.make_weights(synth.ARCHS["full"])
    for name in ("full_mid", "full_late"):
        w = synth.make_weights(synth.ARCHS[name])
        for k, v in full.items():
            if not k.startswith("fusion."):
                np.testing.assert_array_equal(w[k], v)
