"""Shared test helpers: seeded inputs, calibrated weights and stored oracle values."""
import json
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def calib():
    return json.load(open(os.path.join(GOLDEN, "calib.json")))


def weights(arch_name: str, calibrated: bool = True):
    arch = synth.ARCHS[arch_name]
    w = synth.make_weights(arch)
    if calibrated:
        c = calib()[arch_name]
        w = synth.apply_calibration(w, c["scale"], c["shift"])
    return arch, w


def golden(cfg: str, G: int, arch: str = ""):
    """Stored oracle values of a workload config (another architecture: `arch`)."""
    tag = f"_{arch}" if arch and arch != synth.CONFIGS[cfg]["arch"] else ""
    path = os.path.join(GOLDEN, f"{cfg}_G{G}{tag}_oracle.json")
    if not os.path.exists(path):
        return None
    return json.load(open(path))


def golden_scores(cfg: str, G: int, arch: str = ""):
    """Stored oracle scores of poses [0, n) of a workload config: all of them when
    the generator wrote a scores file beside the latents, else the latents' poses."""
    tag = f"_{arch}" if arch and arch != synth.CONFIGS[cfg]["arch"] else ""
    path = os.path.join(GOLDEN, f"{cfg}_G{G}{tag}_scores.json")
    if os.path.exists(path):
        return np.array(json.load(open(path))["score"], np.float64)
    gd = golden(cfg, G, arch)
    return None if gd is None else np.array([p["score"] for p in gd["poses"]], np.float64)


def score_tol(ref):
    """Plain-form bound: |s_gpu - s_oracle| <= 1e-4 * max(1, |s_oracle|) per pose."""
    return 1e-4 * np.maximum(1.0, np.abs(np.asarray(ref)))


# Precision-form bound in pK units (scores are calibrated to a pK-like scale).
BF16_PK_TOL = 2e-2

# Precision-form bound on CNN latents, relative to the largest latent entry.  A
# bfloat16 rounding (unit roundoff u = 2^-8, round to nearest even) adds a relative
# error uniform in [-u, u], rms u / sqrt(3).  A layer rounds at most three things
# on the way to its products: the activation, and (frequency-domain layers) its
# spectrum and the weight spectrum, or (direct layers) the weights.  Independent
# errors through the six conv layers of the full model give an rms relative error
# of sqrt(6 * 3 / 3) u = 2.45 u, with no credit taken for cancellation or for the
# averaging of the pool; float32 accumulation (2^-24) is negligible beside it.
BF16_LATENT_TOL = 2.5 * 2.0 ** -8
