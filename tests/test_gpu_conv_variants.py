"""Every conv kernel variant (tile shape, waves, channel chunking) must give the
oracle's CNN latents: each variant is pinned onto every layer it fits and the
3D-CNN head is compared with the FP64 oracle, including ragged output tiles."""
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


# residual layers at D = 12 (G 24), 16 (G 32) and 20 (G 40): the frequency-domain
# plane kernels are compiled for D = 24, 16 and 12 and take D at run time otherwise
CASES = [("tiny", 24), ("full", 24), ("full", 32), ("full", 40), ("paper", 24), ("paper", 40)]


@pytest.fixture(scope="module")
def cases():
    out = {}
    for arch_name, G in CASES:
        arch, w = weights(arch_name)
        b = synth.make_poses("c1" if G == 24 else "c2", 3)  # odd: a lone pose in two-pose tiles
        cen = np.stack([oracle.pose_center(b.xyz[b.atom_off[p]:b.atom_off[p + 1]][
            b.is_lig[b.atom_off[p]:b.atom_off[p + 1]].astype(bool)]) for p in range(b.n_poses)])
        grids = oracle.splat_batch(b, cen, G)
        want = np.stack([oracle.cnn3d_forward(g, w, arch)[0] for g in grids])
        out[(arch_name, G)] = (arch, w, grids, want)
    return out


@pytest.mark.parametrize("arch_name,G", CASES)
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_every_conv_variant_matches_oracle(cases, arch_name, G, prec):
    import torch
    from paper_2104_04547_amd import Scorer, cfabi
    arch, w, grids, want = cases[(arch_name, G)]
    s = Scorer(arch, w, prec)
    try:
        default = s.variants(G)
        names = cfabi.cf_conv_variant_names()
        tried = 0
        x = torch.from_numpy(grids.astype(np.float32)).cuda()
        if prec == "bf16":
            x = x.to(torch.bfloat16)
        for v in range(len(names)):
            sel = list(default)
            fits = False
            for i in range(len(arch.conv)):
                try:
                    trial = list(sel)
                    trial[i] = v
                    s.set_variants(G, trial)
                    sel = trial
                    fits = True
                except cfabi.CfError:
                    s.set_variants(G, sel)
            if not fits:
                continue
            tried += 1
            _say(f"cf_cnn3d_fwd {prec} arch={arch_name} G={G} variant {v} {names[v]} layers={sel}")
            got = s.cnn3d(x, G).cpu().numpy()
            scale = np.abs(want).max()
            if prec == "fp32":
                np.testing.assert_allclose(got, want, rtol=1e-4, atol=1e-4 * scale, err_msg=names[v])
            else:
                np.testing.assert_allclose(got, want, rtol=BF16_LATENT_TOL, atol=BF16_LATENT_TOL * scale,
                                           err_msg=names[v])
        assert tried >= 2
    finally:
        s.close()


# Stride-1 layers on 32^3 activations (64^3 grids) go past the 32-point transforms
# (32 + k - 1 > 32) and run as overlap-save tiles: 2 x 2 tiles of 16 x 16 outputs per
# plane, each through a window of 16 + k - 1 positions.  A narrow stack covers
# k = 7, 5 and 3, a residual add and 32 / 64 output channels on one pose.
TILE_ARCH = dict(conv=((19, 32, 5, 2, -1), (32, 32, 7, 1, -1), (32, 32, 5, 1, 2), (32, 64, 3, 1, -1)), cnn_dense=0)


@pytest.fixture(scope="module")
def tiled_case():
    import dataclasses
    arch = dataclasses.replace(synth.ARCHS["full"], name="tile_probe", **TILE_ARCH)
    w = synth.make_weights(arch)
    b = synth.make_poses("c4", 1, pose0=5)
    cen = oracle.pose_center(b.xyz[b.is_lig.astype(bool)])[None]
    grids = oracle.splat_batch(b, cen, 64)
    want = np.stack([oracle.cnn3d_forward(g, w, arch)[0] for g in grids])
    return arch, w, grids, want


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_tiled_frequency_domain_layers_at_32cube(tiled_case, prec):
    import torch
    from paper_2104_04547_amd import Scorer, cfabi
    arch, w, grids, want = tiled_case
    s = Scorer(arch, w, prec)
    try:
        names = cfabi.cf_conv_variant_names()
        v = list(s.variants(64))
        assert names[v[1]] == "fft32", [names[i] for i in v]   # the 7^3 layer's default
        v[1:] = [names.index("fft32")] * 3
        s.set_variants(64, v)
        _say(f"cf_cnn3d_fwd {prec} tiled frequency-domain layers, G=64, variants {[names[i] for i in v]}")
        x = torch.from_numpy(grids.astype(np.float32)).cuda()
        if prec == "bf16":
            x = x.to(torch.bfloat16)
        got = s.cnn3d(x, 64).cpu().numpy()
        s.check()
        scale = np.abs(want).max()
        tol = 1e-4 if prec == "fp32" else BF16_LATENT_TOL
        np.testing.assert_allclose(got, want, rtol=tol, atol=tol * scale)
    finally:
        s.close()
