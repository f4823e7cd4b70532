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


def score_tol(ref):
    """Plain-form bound: |s_gpu - s_oracle| <= 1e-4 * max(1, |s_oracle|) per pose."""
    return 1e-4 * np.maximum(1.0, np.abs(np.asarray(ref)))


# Precision-form bound in pK units (scores are calibrated to a pK-like scale).
BF16_PK_TOL = 2e-2
