"""The host C pose generator under AddressSanitizer and UndefinedBehaviorSanitizer:
built with gcc from its source beside a small driver that gives every pose buffers
of exactly the documented sizes, it must run clean and produce the same bytes as the
normal build used by the tests and the benchmark."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _fnv(h, arr):
    b = np.ascontiguousarray(arr).view(np.uint8).ravel()
    for x in b.tolist():
        h = ((h ^ x) * 0x100000001B3) & 0xFFFFFFFFFFFFFFFF
    return h


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("cfg,pose0,n", [("c1", 0, 3), ("c2", 5, 2), ("c4", 7, 2)])
def test_pose_generator_clean_under_sanitizers(tmp_path, cfg, pose0, n):
    exe = str(tmp_path / "posegen_check")
    srcs = [os.path.join(ROOT, "synth", "csrc", "posegen.c"), os.path.join(ROOT, "tests", "csrc", "posegen_check.c")]
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", *srcs, "-o", exe, "-lm"], check=True, capture_output=True, text=True)
    c = synth.CONFIGS[cfg]
    lim = list(c["lim"]) + [0] * (4 - len(c["lim"]))
    r = subprocess.run([exe, "0", str(c["stream"]), str(c["mode"]), *map(str, lim), str(pose0), str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    b = synth.make_poses(cfg, n, pose0=pose0, threads=1)
    h = 0xCBF29CE484222325
    for p in range(n):
        a0, a1 = int(b.atom_off[p]), int(b.atom_off[p + 1])
        h = _fnv(h, b.xyz[a0:a1])
        h = _fnv(h, b.feat[a0:a1])
        h = _fnv(h, b.is_lig[a0:a1])
    assert r.stdout.strip() == f"{h:016x}"
