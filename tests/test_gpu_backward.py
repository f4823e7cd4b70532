"""Backward pass on the GPU (cf_backward, plain form) against the FP64 oracle's
vector-Jacobian products (oracle.score_vjp, pinned by torch autograd and finite
differences in test_oracle_grad.py), through the C ABI.

Bound, per gradient tensor: 2e-4 of its largest entry plus 1e-3 of each entry
(float32 forward and backward, reductions of up to ~10^5 terms), plus twice the
tensor's sensitivity to the ReLU kinks.  The float32 forward (2^-20 fixed-point
grid, float32 convolutions) puts pre-activations within ~1e-6 of the exact ones,
so those closer than that to 0 may take the other side of the ReLU; the oracle
measures how far that moves each gradient by taking its masks at u > +delta and
u > -delta (delta = 4e-6) instead of u > 0.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from helpers import weights

pytestmark = pytest.mark.gpu

RELU_DELTA = 4e-6


def _say(msg):
    print(f"\n[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _oracle_grads(b, w, arch, G, dscore):
    want = oracle.score_vjp(b, w, arch, G, dscore)
    hi = oracle.score_vjp(b, w, arch, G, dscore, relu_margin=RELU_DELTA)
    lo = oracle.score_vjp(b, w, arch, G, dscore, relu_margin=-RELU_DELTA)
    kink = {k: max(np.abs(hi[k] - want[k]).max(), np.abs(lo[k] - want[k]).max()) for k in want}
    return want, kink


def _check_grads(got, want, kink, label):
    assert set(got) == set(want)
    worst = []
    for k in want:
        w = np.asarray(want[k], np.float64)
        g = np.asarray(got[k], np.float64)
        scale = max(np.abs(w).max(), 1e-30)
        err = np.abs(g - w)
        tol = 2e-4 * scale + 1e-3 * np.abs(w) + 2.0 * kink[k]
        worst.append((float((err / tol).max()), k, float(err.max() / scale), float(kink[k] / scale)))
        assert not (err > tol).any(), f"{label} {k}: max err {err.max():.3e} (scale {scale:.3e}, kink {kink[k]:.3e})"
    worst.sort(reverse=True)
    print(f"{label}: worst err/tol {worst[0][0]:.2f} ({worst[0][1]}: err/scale {worst[0][2]:.2e}, "
          f"kink/scale {worst[0][3]:.2e})")


def _run(arch_name, cfg, n, G, seed):
    import torch
    from paper_2104_04547_amd import Scorer, cfabi
    arch, w = weights(arch_name)
    b = synth.make_poses(cfg, n)
    dscore = np.random.default_rng(seed).standard_normal(n)
    s = Scorer(arch, w, "fp32")
    try:
        db = cfabi.DeviceBatch.from_pose_batch(b)
        grad, sc = s.backward(db, G, torch.from_numpy(dscore.astype(np.float32)))
        s.check()
        got = s.unpack_params(grad)
        ref_scores = s.score(db, G).cpu().numpy()
        s.check()
        return arch, w, b, dscore, got, sc.cpu().numpy(), ref_scores
    finally:
        s.close()


@pytest.mark.parametrize("arch_name,cfg,n,G", [("tiny", "c1", 6, 24), ("full", "c1", 2, 24)])
def test_backward_matches_oracle_vjp(arch_name, cfg, n, G):
    _say(f"cf_backward {arch_name} {cfg} poses={n} G={G}")
    arch, w, b, dscore, got, scores, ref_scores = _run(arch_name, cfg, n, G, 3)
    want, kink = _oracle_grads(b, w, arch, G, dscore)
    _check_grads(got, want, kink, f"{arch_name} G={G}")
    # the scores of the backward's own forward are the scoring path's
    np.testing.assert_allclose(scores, ref_scores, rtol=1e-5, atol=1e-5)


def test_backward_chunks_and_determinism():
    # 40 poses: two chunks (32 + 8) accumulated in order; the same call twice is
    # bitwise identical
    import torch
    from paper_2104_04547_amd import Scorer, cfabi
    _say("cf_backward tiny c1 poses=40 G=24, twice")
    arch, w = weights("tiny")
    b = synth.make_poses("c1", 40)
    dscore = np.random.default_rng(7).standard_normal(40)
    s = Scorer(arch, w, "fp32")
    try:
        db = cfabi.DeviceBatch.from_pose_batch(b)
        ds = torch.from_numpy(dscore.astype(np.float32))
        g1, _ = s.backward(db, 24, ds)
        g2, _ = s.backward(db, 24, ds)
        s.check()
        assert torch.equal(g1, g2)
        got = s.unpack_params(g1)
    finally:
        s.close()
    want, kink = _oracle_grads(b, w, arch, 24, dscore)
    _check_grads(got, want, kink, "tiny 40 poses")


def test_backward_refuses_unsupported_forms():
    import torch
    from paper_2104_04547_amd import Scorer, cfabi
    _say("cf_backward unsupported forms")
    b = synth.make_poses("c1", 2)
    ds = torch.ones(2)
    for arch_name, prec in (("tiny", "bf16"), ("paper", "fp32"), ("full_late", "fp32")):
        arch, w = weights(arch_name)
        s = Scorer(arch, w, prec)
        try:
            with pytest.raises(cfabi.CfError) as e:
                s.backward(cfabi.DeviceBatch.from_pose_batch(b), 24, ds)
            assert e.value.code == cfabi.CF_ERR_UNSUPPORTED
        finally:
            s.close()
