"""Thin ctypes binding of libcf.so (include/cf.h): argument marshalling only.

Every function here has the name of the C entry point it wraps and passes device
pointers (``tensor.data_ptr()``) and a HIP stream handle straight through; every
step of the scoring path runs in the library's HIP kernels.  PyTorch supplies
device memory and streams, nothing else.  If the library is not built, importing
this module raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import struct
from typing import Dict, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcf.so")

CF_OK, CF_ERR_INVALID_ARG, CF_ERR_CAPACITY, CF_ERR_OOM, CF_ERR_HIP, CF_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
CF_ERR_CANCELLED = -6
CF_PREC_FP32, CF_PREC_BF16 = 0, 1
CF_NCH = 19
CF_MAX_POSE_ATOMS = 4096
CF_MODEL_MAGIC = 0x314D4643

EXPORTS = ["cf_create", "cf_destroy", "cf_pose_centers", "cf_voxelize", "cf_build_graphs", "cf_cnn3d_fwd",
           "cf_sgcnn_fwd", "cf_score_poses", "cf_stream_status", "cf_last_error", "cf_model_info",
           "cf_autotune", "cf_conv_variants", "cf_timing_enable", "cf_timing_read",
           "cf_engine_create", "cf_engine_submit", "cf_engine_poll", "cf_engine_wait_all", "cf_engine_info",
           "cf_engine_last_error", "cf_engine_destroy", "cf_engine_cancel", "cf_set_conv_variants", "cf_conv_variant_count",
           "cf_conv_variant_name", "cf_compound_max", "cf_top_k", "cf_fusion_fwd",
           "cf_top_k_noalloc", "cf_backward"]


HEAD_KINDS = {"coherent": 0, "mid": 1, "late": 2}   # cf_head_kind


class CfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"cf status {code}: {msg}")
        self.code = code


class cf_pose_batch(ctypes.Structure):
    _fields_ = [("n_poses", ctypes.c_int32), ("n_atoms", ctypes.c_int32), ("atom_off", ctypes.c_void_p),
                ("xyz", ctypes.c_void_p), ("feat", ctypes.c_void_p), ("is_lig", ctypes.c_void_p),
                ("center", ctypes.c_void_p)]


class cf_csr(ctypes.Structure):
    _fields_ = [("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("capacity", ctypes.c_int64)]


class cf_model_desc(ctypes.Structure):
    _fields_ = [("magic", ctypes.c_uint32), ("n_ch", ctypes.c_int32), ("n_conv", ctypes.c_int32),
                ("conv", (ctypes.c_int32 * 5) * 8), ("bn", ctypes.c_int32), ("cnn_dense", ctypes.c_int32),
                ("H", ctypes.c_int32), ("K_c", ctypes.c_int32), ("K_n", ctypes.c_int32),
                ("r_cov_u", ctypes.c_int32), ("r_nc_u", ctypes.c_int32), ("fusion_hidden", ctypes.c_int32),
                ("head", ctypes.c_int32), ("fusion_layers", ctypes.c_int32), ("fusion_residual", ctypes.c_int32),
                ("sg_dense", ctypes.c_int32 * 2), ("cnn_dense2", ctypes.c_int32), ("H_nc", ctypes.c_int32)]


class cf_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 64), ("launches", ctypes.c_int32), ("total_ms", ctypes.c_double),
                ("flop", ctypes.c_double), ("bytes", ctypes.c_double)]


class cf_engine_config(ctypes.Structure):
    _fields_ = [("n_slots", ctypes.c_int32), ("slot_poses", ctypes.c_int32), ("slot_atoms", ctypes.c_int64),
                ("hbm_budget_bytes", ctypes.c_int64), ("use_graphs", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libcf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run python -m paper_2104_04547_amd.build")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    pb = ctypes.POINTER(cf_pose_batch)
    pc = ctypes.POINTER(cf_csr)
    sig = {
        "cf_create": ([vp, ctypes.c_size_t, ctypes.c_int, i64, ctypes.POINTER(vp)], ctypes.c_int),
        "cf_destroy": ([vp], None),
        "cf_pose_centers": ([vp, pb, vp, vp], ctypes.c_int),
        "cf_voxelize": ([vp, pb, ctypes.c_int, vp, vp], ctypes.c_int),
        "cf_build_graphs": ([vp, pb, pc, pc, vp], ctypes.c_int),
        "cf_cnn3d_fwd": ([vp, vp, i32, ctypes.c_int, vp, vp], ctypes.c_int),
        "cf_sgcnn_fwd": ([vp, pb, pc, pc, vp, vp], ctypes.c_int),
        "cf_score_poses": ([vp, pb, ctypes.c_int, vp, vp], ctypes.c_int),
        "cf_stream_status": ([vp, vp, ctypes.POINTER(i64), ctypes.POINTER(i64)], ctypes.c_int),
        "cf_last_error": ([], ctypes.c_char_p),
        "cf_model_info": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64),
                           ctypes.POINTER(i32)], ctypes.c_int),
        "cf_autotune": ([vp, ctypes.c_int, i32, vp], ctypes.c_int),
        "cf_conv_variants": ([vp, ctypes.c_int, ctypes.POINTER(i32), i32], ctypes.c_int),
        "cf_timing_enable": ([vp, ctypes.c_int], ctypes.c_int),
        "cf_timing_read": ([vp, ctypes.POINTER(cf_kernel_stat), i32, ctypes.POINTER(i32)], ctypes.c_int),
        "cf_engine_create": ([vp, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(cf_engine_config),
                              ctypes.POINTER(vp)], ctypes.c_int),
        "cf_engine_submit": ([vp, i32, vp, vp, vp, vp, i32, ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "cf_engine_poll": ([vp, ctypes.c_uint64, vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)],
                           ctypes.c_int),
        "cf_engine_wait_all": ([vp], ctypes.c_int),
        "cf_engine_cancel": ([vp, ctypes.c_uint64, ctypes.POINTER(i32)], ctypes.c_int),
        "cf_engine_info": ([vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64)],
                           ctypes.c_int),
        "cf_engine_last_error": ([vp], ctypes.c_char_p),
        "cf_engine_destroy": ([vp], None),
        "cf_set_conv_variants": ([vp, ctypes.c_int, ctypes.POINTER(i32), i32], ctypes.c_int),
        "cf_conv_variant_count": ([], ctypes.c_int),
        "cf_conv_variant_name": ([i32], ctypes.c_char_p),
        "cf_compound_max": ([vp, vp, i32, vp, i32, vp, vp, vp], ctypes.c_int),
        "cf_top_k": ([vp, vp, i32, i32, vp, vp, vp], ctypes.c_int),
        "cf_top_k_noalloc": ([vp, i32, i32, vp, vp, vp], ctypes.c_int),
        "cf_backward": ([vp, ctypes.POINTER(cf_pose_batch), ctypes.c_int, vp, vp, vp, vp], ctypes.c_int),
        "cf_fusion_fwd": ([vp, vp, vp, i32, vp, vp], ctypes.c_int),
    }
    missing = set(EXPORTS) - set(sig)
    if missing:   # an undeclared signature would pass pointers as 32-bit ints
        raise ImportError(f"no ctypes signature for {sorted(missing)}")
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != CF_OK:
        raise CfError(rc, load().cf_last_error().decode(errors="replace"))


# ------------------------------------------------------------------ model blob

def model_desc(arch) -> cf_model_desc:
    d = cf_model_desc()
    d.magic = CF_MODEL_MAGIC
    d.n_ch = arch.n_ch
    d.n_conv = len(arch.conv)
    for i, row in enumerate(arch.conv):
        for j, v in enumerate(row):
            d.conv[i][j] = int(v)
    d.bn = int(arch.bn)
    d.cnn_dense = arch.cnn_dense
    d.H, d.K_c, d.K_n = arch.H, arch.K_c, arch.K_n
    d.r_cov_u, d.r_nc_u = arch.r_cov_u, arch.r_nc_u
    d.fusion_hidden = arch.fusion_hidden
    d.head = HEAD_KINDS[arch.head]
    d.fusion_layers = arch.n_fusion
    d.fusion_residual = int(arch.fusion_residual)
    if len(arch.sg_dense) > 2:
        raise ValueError("at most two SG-CNN dense layers")
    for j, v in enumerate(arch.sg_dense):
        d.sg_dense[j] = int(v)
    d.cnn_dense2 = arch.cnn_dense2
    d.H_nc = arch.H_nc
    return d


def blob_param_order(arch):
    """Parameter names in the order the blob stores them (see include/cf.h)."""
    names = []
    for i in range(len(arch.conv)):
        names += [f"conv{i}.w", f"conv{i}.b"]
        if arch.bn:
            names += [f"bn{i}.gamma", f"bn{i}.beta", f"bn{i}.mean", f"bn{i}.var"]
    if arch.cnn_dense:
        names += ["cnn_dense.w", "cnn_dense.b"]
    if arch.cnn_dense2:
        names += ["cnn_dense2.w", "cnn_dense2.b"]
    names += ["sg.embed.w", "sg.embed.b"]
    for stage, K in (("cov", arch.K_c), ("nc", arch.K_n)):
        if stage == "nc" and arch.H_nc:
            names += ["sg.mid.gate.w", "sg.mid.gate.b", "sg.mid.val.w", "sg.mid.val.b", "sg.embed2.w", "sg.embed2.b"]
        names += [f"sg.{stage}.msg{t}.w" for t in range(K)]
        names += [f"sg.{stage}.gru.w_ih", f"sg.{stage}.gru.w_hh", f"sg.{stage}.gru.b_ih", f"sg.{stage}.gru.b_hh"]
    names += ["sg.gate.w", "sg.gate.b", "sg.val.w", "sg.val.b"]
    if arch.head == "late":
        names += ["late.cnn_out.w", "late.cnn_out.b"]
        for j in range(len(arch.sg_dense)):
            names += [f"late.sg_dense{j}.w", f"late.sg_dense{j}.b"]
        return names + ["late.sg_out.w", "late.sg_out.b"]
    if arch.head == "mid":
        names += ["mid.cnn.w", "mid.cnn.b", "mid.sg.w", "mid.sg.b"]
    for l in range(arch.n_fusion - 1):
        n = "fusion.hidden" if l == 0 else f"fusion.hidden{l}"
        names += [n + ".w", n + ".b"]
    return names + ["fusion.out.w", "fusion.out.b"]


def pack_model(arch, params: Dict[str, np.ndarray]) -> bytes:
    """Serialise an architecture + named float32 parameters into the cf.h blob."""
    d = model_desc(arch)
    parts = [bytes(d)]
    for name in blob_param_order(arch):
        parts.append(np.ascontiguousarray(params[name], dtype="<f4").tobytes())
    return b"".join(parts)


# ------------------------------------------------------------------ entry points

def cf_create(blob: bytes, precision: int, hbm_budget_bytes: int = 0) -> int:
    lib = load()
    out = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(lib.cf_create(ctypes.cast(buf, ctypes.c_void_p), len(blob), precision, hbm_budget_bytes,
                         ctypes.byref(out)))
    return out.value


def cf_destroy(ctx: int) -> None:
    load().cf_destroy(ctx)


def cf_pose_centers(ctx, batch: cf_pose_batch, center_out_ptr: int, stream: int = 0):
    _check(load().cf_pose_centers(ctx, ctypes.byref(batch), center_out_ptr, stream))


def cf_voxelize(ctx, batch: cf_pose_batch, G: int, grid_out_ptr: int, stream: int = 0):
    _check(load().cf_voxelize(ctx, ctypes.byref(batch), G, grid_out_ptr, stream))


def cf_build_graphs(ctx, batch: cf_pose_batch, cov: cf_csr, nc: cf_csr, stream: int = 0):
    _check(load().cf_build_graphs(ctx, ctypes.byref(batch), ctypes.byref(cov), ctypes.byref(nc), stream))


def cf_cnn3d_fwd(ctx, grid_ptr: int, n_poses: int, G: int, cnn_latent_ptr: int, stream: int = 0):
    _check(load().cf_cnn3d_fwd(ctx, grid_ptr, n_poses, G, cnn_latent_ptr, stream))


def cf_sgcnn_fwd(ctx, batch: cf_pose_batch, cov: cf_csr, nc: cf_csr, sg_latent_ptr: int, stream: int = 0):
    _check(load().cf_sgcnn_fwd(ctx, ctypes.byref(batch), ctypes.byref(cov), ctypes.byref(nc), sg_latent_ptr,
                               stream))


def cf_fusion_fwd(ctx, cnn_latent_ptr: int, sg_latent_ptr: int, n_poses: int, scores_ptr: int, stream: int = 0):
    _check(load().cf_fusion_fwd(ctx, cnn_latent_ptr, sg_latent_ptr, n_poses, scores_ptr, stream))


def cf_score_poses(ctx, batch: cf_pose_batch, G: int, scores_ptr: int, stream: int = 0):
    _check(load().cf_score_poses(ctx, ctypes.byref(batch), G, scores_ptr, stream))


def cf_backward(ctx, batch: cf_pose_batch, G: int, dscore_ptr: int, grad_ptr: int, scores_ptr, stream: int = 0):
    _check(load().cf_backward(ctx, ctypes.byref(batch), G, dscore_ptr, grad_ptr, scores_ptr, stream))


def cf_stream_status(ctx, stream: int = 0):
    """Returns (status, need_cov, need_nc); never raises for device-side errors."""
    nc_, nn_ = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = load().cf_stream_status(ctx, stream, ctypes.byref(nc_), ctypes.byref(nn_))
    return rc, nc_.value, nn_.value


def cf_last_error() -> str:
    return load().cf_last_error().decode(errors="replace")


def cf_model_info(ctx):
    lc, ls, npar, prec = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
    _check(load().cf_model_info(ctx, ctypes.byref(lc), ctypes.byref(ls), ctypes.byref(npar), ctypes.byref(prec)))
    return lc.value, ls.value, npar.value, prec.value


def cf_autotune(ctx, G: int, n_poses: int, stream: int = 0):
    _check(load().cf_autotune(ctx, G, n_poses, stream))


def cf_conv_variants(ctx, G: int, n_layers: int):
    arr = (ctypes.c_int32 * n_layers)()
    _check(load().cf_conv_variants(ctx, G, arr, n_layers))
    return list(arr)


def cf_set_conv_variants(ctx, G: int, variants):
    arr = (ctypes.c_int32 * len(variants))(*variants)
    _check(load().cf_set_conv_variants(ctx, G, arr, len(variants)))


def cf_conv_variant_names():
    lib = load()
    return [lib.cf_conv_variant_name(i).decode() for i in range(lib.cf_conv_variant_count())]


def cf_compound_max(ctx, scores_ptr: int, n_scores: int, off_ptr: int, n_compounds: int, best_ptr: int,
                    best_idx_ptr: int, stream: int = 0):
    _check(load().cf_compound_max(ctx, scores_ptr, n_scores, off_ptr, n_compounds, best_ptr, best_idx_ptr, stream))


def cf_top_k(ctx, values_ptr: int, n: int, k: int, idx_ptr: int, val_ptr, stream: int = 0):
    _check(load().cf_top_k(ctx, values_ptr, n, k, idx_ptr, val_ptr, stream))


def cf_top_k_noalloc(values_ptr: int, n: int, k: int, idx_ptr: int, val_ptr, stream: int = 0):
    _check(load().cf_top_k_noalloc(values_ptr, n, k, idx_ptr, val_ptr, stream))


CF_TIMING_EVENTS, CF_TIMING_ROCTX = 1, 2


def cf_timing_enable(ctx, enable: bool = True, roctx: bool = False):
    """Per-launch event timing and / or roctx stage ranges (see cf.h)."""
    _check(load().cf_timing_enable(ctx, (CF_TIMING_EVENTS if enable else 0) | (CF_TIMING_ROCTX if roctx else 0)))


def cf_timing_read(ctx):
    """{kernel: dict(launches, total_ms, flop, bytes)}; clears the accumulated entries."""
    arr = (cf_kernel_stat * 64)()
    n = ctypes.c_int32(0)
    _check(load().cf_timing_read(ctx, arr, 64, ctypes.byref(n)))
    return {arr[i].name.decode(): dict(launches=arr[i].launches, total_ms=arr[i].total_ms, flop=arr[i].flop,
                                       bytes=arr[i].bytes) for i in range(min(n.value, 64))}


def cf_engine_create(blob: bytes, precision: int, n_slots: int = 4, slot_poses: int = 512,
                     slot_atoms: int = 512 * 1600, hbm_budget_bytes: int = 0, use_graphs: bool = True) -> int:
    cfg = cf_engine_config(n_slots, slot_poses, slot_atoms, hbm_budget_bytes, int(use_graphs), 0)
    out = ctypes.c_void_p()
    buf = ctypes.create_string_buffer(blob, len(blob))
    _check(load().cf_engine_create(ctypes.cast(buf, ctypes.c_void_p), len(blob), precision, ctypes.byref(cfg),
                                   ctypes.byref(out)))
    return out.value


def cf_engine_submit(eng, atom_off, xyz, feat, is_lig, G: int) -> int:
    """Host numpy arrays (copied by the engine before this returns)."""
    t = ctypes.c_uint64(0)
    atom_off = np.ascontiguousarray(atom_off, dtype=np.int32)
    xyz = np.ascontiguousarray(xyz, dtype=np.int32)
    feat = np.ascontiguousarray(feat, dtype=np.float32)
    is_lig = np.ascontiguousarray(is_lig, dtype=np.uint8)
    rc = load().cf_engine_submit(eng, len(atom_off) - 1, atom_off.ctypes.data, xyz.ctypes.data, feat.ctypes.data,
                                 is_lig.ctypes.data, G, ctypes.byref(t))
    if rc != CF_OK:
        raise CfError(rc, load().cf_engine_last_error(eng).decode(errors="replace"))
    return t.value


def cf_engine_poll(eng, ticket: int, n_poses: int):
    """(done, scores or None, latency_ms or None); raises if the request failed."""
    out = np.empty(n_poses, dtype=np.float32)
    done = ctypes.c_int32(0)
    lat = ctypes.c_double(0.0)
    rc = load().cf_engine_poll(eng, ticket, out.ctypes.data, ctypes.byref(done), ctypes.byref(lat))
    if rc != CF_OK:
        raise CfError(rc, load().cf_engine_last_error(eng).decode(errors="replace"))
    return (True, out, lat.value) if done.value else (False, None, None)


def cf_engine_cancel(eng, ticket: int) -> bool:
    """True if the request was still queued and is now withdrawn."""
    c = ctypes.c_int32(0)
    rc = load().cf_engine_cancel(eng, ticket, ctypes.byref(c))
    if rc != CF_OK:
        raise CfError(rc, load().cf_engine_last_error(eng).decode(errors="replace"))
    return bool(c.value)


def cf_engine_wait_all(eng):
    _check(load().cf_engine_wait_all(eng))


def cf_engine_info(eng):
    a, b, c, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(load().cf_engine_info(eng, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c), ctypes.byref(d)))
    return dict(poses_done=a.value, batches=b.value, graph_replays=c.value, queued_poses=d.value)


def cf_engine_destroy(eng):
    load().cf_engine_destroy(eng)


# ------------------------------------------------------------------ torch helpers

class DeviceBatch:
    """Holds a pose batch's device tensors and the matching cf_pose_batch."""

    def __init__(self, atom_off, xyz, feat, is_lig, center=None):
        import torch
        dev = torch.device("cuda")
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dtype=dt).contiguous()
        self.atom_off = t(atom_off, torch.int32)
        self.xyz = t(xyz, torch.int32)
        self.feat = t(feat, torch.float32)
        self.is_lig = t(is_lig, torch.uint8)
        self.center = None if center is None else t(center, torch.int32)
        self.n_poses = int(len(atom_off) - 1)
        self.n_atoms = int(atom_off[-1])
        self.c = cf_pose_batch(self.n_poses, self.n_atoms, self.atom_off.data_ptr(), self.xyz.data_ptr(),
                               self.feat.data_ptr(), self.is_lig.data_ptr(),
                               None if self.center is None else self.center.data_ptr())

    @classmethod
    def from_pose_batch(cls, b, center=None):
        return cls(b.atom_off, b.xyz, b.feat, b.is_lig, center)


def current_stream() -> int:
    import torch
    return torch.cuda.current_stream().cuda_stream
