"""FP64 CPU oracle for Coherent Fusion pose scoring -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import or run anything in this package.  The scoring library never calls it, and
it shares no code with the HIP path (no kernels, headers, helpers, tables or
pre/post-processing); both sides consume only the seeded inputs of `synth`.

Every stage is the plain definition written out in float64 (float32 inputs are
widened exactly), following the paper's pipeline (Sec. 1, 2.1-2.2, 3.3; Fig. 1;
Tables II-V) and the readings listed in the design notes where the paper defers
details to its predecessor.  Pins for each function live in tests/test_oracle_*.py.
"""
from .cf_oracle import (U_PER_A, SPLAT_RCUT_U, SPLAT_TWO_SIGMA2_U2, SELU_LAMBDA, SELU_ALPHA,
                        pose_center, voxel_center, splat_pose, splat_batch, conv3d, batchnorm,
                        cnn3d_forward, radius_graph_pose, radius_graph_batch, gru_cell,
                        sgcnn_pose, sgcnn_batch, selu, fusion_head, late_fusion, score_pose,
                        score_batch, compound_best, top_k)
from .cf_grad import (conv3d_vjp, batchnorm_vjp, cnn3d_vjp, aggregate_vjp, gru_cell_vjp, sgcnn_vjp,
                      fusion_head_vjp, score_vjp)

__all__ = ["U_PER_A", "SPLAT_RCUT_U", "SPLAT_TWO_SIGMA2_U2", "SELU_LAMBDA", "SELU_ALPHA",
           "pose_center", "voxel_center", "splat_pose", "splat_batch", "conv3d", "batchnorm",
           "cnn3d_forward", "radius_graph_pose", "radius_graph_batch", "gru_cell", "sgcnn_pose",
           "sgcnn_batch", "selu", "fusion_head", "late_fusion", "score_pose", "score_batch",
           "compound_best", "top_k", "conv3d_vjp", "batchnorm_vjp", "cnn3d_vjp", "aggregate_vjp",
           "gru_cell_vjp", "sgcnn_vjp", "fusion_head_vjp", "score_vjp"]
