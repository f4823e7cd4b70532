"""Seeded synthetic pose batches (ragged, CSR-packed by `atom_off`).

The generator itself is C (`csrc/posegen.c`, compiled with gcc on first use);
this module sizes poses, runs the generator over a thread pool (ctypes releases
the GIL) and packs the result.  Atoms of pose p are rows atom_off[p] ..
atom_off[p+1]-1, ligand atoms first.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor
from typing import List, Optional, Sequence

import numpy as np

from .model import CONFIGS

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csrc", "posegen.c")
_LIB_PATH = os.path.join(_HERE, "_posegen.so")
_lib = None
_lock = threading.Lock()


def build(force: bool = False) -> str:
    """Compile the generator with gcc (no fast-math: results must be reproducible)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            lib.cfgen_pose.restype = ctypes.c_double
            lib.cfgen_pose.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int,
                                       ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
            lib.cfgen_work_bytes.restype = ctypes.c_size_t
            lib.cfgen_work_bytes.argtypes = [ctypes.c_int]
            lib.cfgen_pose_sizes.restype = None
            lib.cfgen_pose_sizes.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                             ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
            _lib = lib
    return _lib


@dataclasses.dataclass
class PoseBatch:
    """A ragged batch of poses.

    atom_off [P+1] int32, xyz [N,3] int32 (units 2^-10 A), feat [N,19] float32,
    is_lig [N] uint8, n_lig [P] int32.  Grid centres are not part of the batch:
    the scorer derives them from the ligand atoms (or the caller passes its own).
    """
    atom_off: np.ndarray
    xyz: np.ndarray
    feat: np.ndarray
    is_lig: np.ndarray
    n_lig: np.ndarray

    @property
    def n_poses(self) -> int:
        return len(self.atom_off) - 1

    @property
    def n_atoms(self) -> int:
        return int(self.atom_off[-1])

    def pose(self, p: int) -> "PoseBatch":
        return self.select([p])

    def select(self, idx: Sequence[int]) -> "PoseBatch":
        parts = [slice(int(self.atom_off[p]), int(self.atom_off[p + 1])) for p in idx]
        n = np.array([s.stop - s.start for s in parts], dtype=np.int64)
        off = np.zeros(len(idx) + 1, dtype=np.int32)
        off[1:] = np.cumsum(n)
        cat = lambda a: np.concatenate([a[s] for s in parts]) if parts else a[:0]
        return PoseBatch(off, np.ascontiguousarray(cat(self.xyz)), np.ascontiguousarray(cat(self.feat)),
                         np.ascontiguousarray(cat(self.is_lig)),
                         np.ascontiguousarray(self.n_lig[list(idx)]))


def concat_batches(bs: Sequence[PoseBatch]) -> PoseBatch:
    n = np.concatenate([np.diff(b.atom_off) for b in bs])
    off = np.zeros(len(n) + 1, dtype=np.int32)
    off[1:] = np.cumsum(n)
    return PoseBatch(off, np.concatenate([b.xyz for b in bs]), np.concatenate([b.feat for b in bs]),
                     np.concatenate([b.is_lig for b in bs]), np.concatenate([b.n_lig for b in bs]))


def pose_sizes(config: str, n_poses: int, pose0: int = 0, seed: int = 0):
    cfg = CONFIGS[config]
    lib = _load()
    lim = np.array(cfg["lim"] + (0,) * (4 - len(cfg["lim"])), dtype=np.int32)
    nl = np.zeros(n_poses, dtype=np.int32)
    npk = np.zeros(n_poses, dtype=np.int32)
    lib.cfgen_pose_sizes(seed, cfg["stream"], pose0, n_poses, cfg["mode"], lim.ctypes.data,
                         nl.ctypes.data, npk.ctypes.data)
    return nl, npk


def make_poses(config: str, n_poses: int, pose0: int = 0, seed: int = 0,
               threads: Optional[int] = None, r_in: float = 4.0, r_out: float = 10.0,
               jam: int = 2000) -> PoseBatch:
    """Poses pose0 .. pose0+n_poses-1 of a workload config (each from its own stream)."""
    cfg = CONFIGS[config]
    lib = _load()
    nl, npk = pose_sizes(config, n_poses, pose0, seed)
    n = (nl + npk).astype(np.int64)
    off = np.zeros(n_poses + 1, dtype=np.int64)
    off[1:] = np.cumsum(n)
    N = int(off[-1])
    xyz = np.zeros((N, 3), dtype=np.int32)
    feat = np.zeros((N, 19), dtype=np.float32)
    is_lig = np.zeros(N, dtype=np.uint8)
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    threads = max(1, min(threads, n_poses))
    failed: List[int] = []

    def work(tid: int):
        wb = np.empty(lib.cfgen_work_bytes(int(n.max())) // 8 + 8, dtype=np.float64)
        for p in range(tid, n_poses, threads):
            a = int(off[p])
            r = lib.cfgen_pose(seed, cfg["stream"], pose0 + p, int(nl[p]), int(npk[p]), r_in, r_out, jam,
                               wb.ctypes.data, xyz[a:].ctypes.data, feat[a:].ctypes.data,
                               is_lig[a:].ctypes.data)
            if r < 0:
                failed.append(p)

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(work, range(threads)))
    if failed:
        raise RuntimeError(f"pose generator failed for poses {failed[:8]}")
    return PoseBatch(off.astype(np.int32), xyz, feat, is_lig, nl)
