"""Convenience wrapper over the C ABI: owns a context and allocates outputs with torch.

All computation happens in libcf.so; this class only allocates output tensors on
the current device and forwards pointers and the current HIP stream.
"""
from __future__ import annotations

from typing import Dict, Optional, Tuple

import numpy as np

from . import cfabi


class Scorer:
    def __init__(self, arch, params: Dict[str, np.ndarray], precision: str = "bf16", hbm_budget_bytes: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Scorer needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.arch = arch
        self.precision = precision
        self.param_shapes = {k: np.shape(v) for k, v in params.items()}
        prec = {"bf16": cfabi.CF_PREC_BF16, "fp32": cfabi.CF_PREC_FP32}[precision]
        self.ctx = cfabi.cf_create(cfabi.pack_model(arch, params), prec, hbm_budget_bytes)
        self.lc, self.H, self.n_params, _ = cfabi.cf_model_info(self.ctx)

    # -- lifetime
    def close(self):
        if self.ctx:
            cfabi.cf_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def grid_dtype(self):
        import torch
        return torch.bfloat16 if self.precision == "bf16" else torch.float32

    def _stream(self) -> int:
        return cfabi.current_stream()

    # -- entry points
    def centers(self, db: "cfabi.DeviceBatch"):
        import torch
        out = torch.empty((db.n_poses, 3), dtype=torch.int32, device="cuda")
        cfabi.cf_pose_centers(self.ctx, db.c, out.data_ptr(), self._stream())
        return out

    def voxelize(self, db, G: int):
        import torch
        out = torch.empty((db.n_poses, G, G, G, cfabi.CF_NCH), dtype=self.grid_dtype, device="cuda")
        cfabi.cf_voxelize(self.ctx, db.c, G, out.data_ptr(), self._stream())
        return out

    def build_graphs(self, db, cov_capacity: Optional[int] = None, nc_capacity: Optional[int] = None):
        import torch
        n = db.n_atoms
        cov_capacity = 16 * n if cov_capacity is None else cov_capacity
        nc_capacity = 96 * n if nc_capacity is None else nc_capacity
        t = dict(cov_row=torch.empty(n + 1, dtype=torch.int32, device="cuda"),
                 cov_col=torch.empty(max(cov_capacity, 1), dtype=torch.int32, device="cuda"),
                 nc_row=torch.empty(n + 1, dtype=torch.int32, device="cuda"),
                 nc_col=torch.empty(max(nc_capacity, 1), dtype=torch.int32, device="cuda"))
        cov = cfabi.cf_csr(t["cov_row"].data_ptr(), t["cov_col"].data_ptr(), cov_capacity)
        nc = cfabi.cf_csr(t["nc_row"].data_ptr(), t["nc_col"].data_ptr(), nc_capacity)
        cfabi.cf_build_graphs(self.ctx, db.c, cov, nc, self._stream())
        t["cov"], t["nc"] = cov, nc
        return t

    def cnn3d(self, grid, G: int):
        import torch
        P = grid.shape[0]
        out = torch.empty((P, self.lc), dtype=torch.float32, device="cuda")
        cfabi.cf_cnn3d_fwd(self.ctx, grid.data_ptr(), P, G, out.data_ptr(), self._stream())
        return out

    def sgcnn(self, db, graphs):
        import torch
        out = torch.empty((db.n_poses, self.H), dtype=torch.float32, device="cuda")
        cfabi.cf_sgcnn_fwd(self.ctx, db.c, graphs["cov"], graphs["nc"], out.data_ptr(), self._stream())
        return out

    def score(self, db, G: int, out=None):
        import torch
        if out is None:
            out = torch.empty(db.n_poses, dtype=torch.float32, device="cuda")
        cfabi.cf_score_poses(self.ctx, db.c, G, out.data_ptr(), self._stream())
        return out

    def backward(self, db, G: int, dscore, with_scores: bool = True):
        """Gradients of sum_p dscore[p] * score_p w.r.t. every blob parameter
        (cf_backward, plain form): a device vector in blob order, and the scores."""
        import torch
        grad = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        scores = torch.empty(db.n_poses, dtype=torch.float32, device="cuda") if with_scores else None
        dscore = dscore.to(device="cuda", dtype=torch.float32).contiguous()
        cfabi.cf_backward(self.ctx, db.c, G, dscore.data_ptr(), grad.data_ptr(),
                          scores.data_ptr() if scores is not None else None, self._stream())
        return grad, scores

    def unpack_params(self, vec) -> Dict[str, np.ndarray]:
        """A blob-ordered parameter vector (host or device) as named arrays."""
        v = vec.detach().cpu().numpy() if hasattr(vec, "detach") else np.asarray(vec)
        out, o = {}, 0
        for name in cfabi.blob_param_order(self.arch):
            shape = self.param_shapes[name]
            k = int(np.prod(shape)) if len(shape) else 1
            out[name] = v[o:o + k].reshape(shape)
            o += k
        assert o == v.size, "vector length does not match the model"
        return out

    def status(self) -> Tuple[int, int, int]:
        return cfabi.cf_stream_status(self.ctx, self._stream())

    def check(self):
        rc, nc_, nn_ = self.status()
        if rc != cfabi.CF_OK:
            raise cfabi.CfError(rc, cfabi.cf_last_error() + f" (need cov={nc_}, nc={nn_})")

    def autotune(self, G: int, n_poses: int):
        cfabi.cf_autotune(self.ctx, G, n_poses, self._stream())
        return cfabi.cf_conv_variants(self.ctx, G, len(self.arch.conv))

    def variants(self, G: int):
        return cfabi.cf_conv_variants(self.ctx, G, len(self.arch.conv))

    def fusion(self, cnn_latent, sg_latent):
        """Fusion head alone: one pK per pose from device float32 latents."""
        import torch
        n = cnn_latent.shape[0]
        out = torch.empty(n, dtype=torch.float32, device="cuda")
        cfabi.cf_fusion_fwd(self.ctx, cnn_latent.contiguous().data_ptr(), sg_latent.contiguous().data_ptr(), n,
                            out.data_ptr(), self._stream())
        return out

    def compound_max(self, scores, compound_off):
        """Best score and pose index per compound segment (device tensors)."""
        import torch
        off = compound_off.to(device="cuda", dtype=torch.int32).contiguous()
        n = off.numel() - 1
        best = torch.empty(n, dtype=torch.float32, device="cuda")
        idx = torch.empty(n, dtype=torch.int32, device="cuda")
        cfabi.cf_compound_max(self.ctx, scores.data_ptr(), scores.numel(), off.data_ptr(), n, best.data_ptr(),
                              idx.data_ptr(), self._stream())
        return best, idx

    def top_k(self, values, k: int):
        import torch
        idx = torch.empty(k, dtype=torch.int32, device="cuda")
        val = torch.empty(k, dtype=torch.float32, device="cuda")
        cfabi.cf_top_k(self.ctx, values.data_ptr(), values.numel(), k, idx.data_ptr(), val.data_ptr(), self._stream())
        return idx, val

    def set_variants(self, G: int, variants):
        cfabi.cf_set_conv_variants(self.ctx, G, list(variants))
