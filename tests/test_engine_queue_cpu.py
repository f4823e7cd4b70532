"""Serving engine request queue on the CPU: arrival-order packing by grid size,
pose / atom limits and cancellation of queued requests (the host-only queue the
engine's scheduler uses, built here with g++ without HIP)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_request_queue_packing_and_cancel(tmp_path):
    exe = str(tmp_path / "queue_test")
    src = os.path.join(ROOT, "tests", "csrc", "queue_test.cpp")
    inc = os.path.join(ROOT, "paper_2104_04547_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined", "-I", inc, src,
                    "-o", exe], check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.strip() == "OK", r.stdout + r.stderr
