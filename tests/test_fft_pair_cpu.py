"""Host check of the 32-point transforms that two lanes share in the frequency-domain
conv kernels (decimation in time and in frequency, both directions): built with g++
from the kernels' own header, the two lanes run one after the other with an explicit
exchange and are compared with the one-lane transform and with a direct DFT."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_lane_pair_fft32_matches_dft(tmp_path):
    exe = str(tmp_path / "fft_pair_test")
    src = os.path.join(ROOT, "tests", "csrc", "fft_pair_test.cpp")
    inc = os.path.join(ROOT, "paper_2104_04547_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Wno-unknown-pragmas", "-fsanitize=address,undefined",
                    "-I", inc, src, "-o", exe], check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and r.stdout.strip() == "OK", r.stdout + r.stderr
