"""Seeded synthetic inputs for the Coherent Fusion pose scorer.

This package only *generates inputs*: docked-pose stand-ins (atoms, fixed-point
coordinates, 19 feature channels) and random model weights.  It holds none of the
scoring method's arithmetic; both the FP64 oracle and the HIP path consume the
arrays it returns.
"""
from .model import ARCHS, CONFIGS, ModelArch, make_weights, apply_calibration, n_params
from .poses import PoseBatch, make_poses, pose_sizes, concat_batches

__all__ = ["ARCHS", "CONFIGS", "ModelArch", "make_weights", "apply_calibration", "n_params",
           "PoseBatch", "make_poses", "pose_sizes", "concat_batches"]
