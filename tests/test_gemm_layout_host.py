"""The matrix-core engine's lane layout (csrc/gemm_layout.h: which sample,
bin and DFT-matrix entry every lane holds in each of the four products, the
twiddle exponents and the kept output rows), run through a float64 host model
of the real 16x16x32 products and checked against a direct overlap-save block
(DFT, H_R of eq. (6), inverse DFT with 1/N, phase as a delay of D samples):
an index, sign or permutation slip gives an O(1) error."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2406_14116_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_gemm_layout_matches_direct_block(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")):
        pytest.skip("g++ or HIP headers missing")
    exe = str(tmp_path / "check")
    subprocess.run([gxx, "-O1", "-std=c++20", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
                    "-I", CSRC, os.path.join(os.path.dirname(__file__), "gemm_layout_check.cpp"), "-o", exe],
                   check=True)
    worst = float(subprocess.run([exe], check=True, capture_output=True, text=True).stdout)
    assert worst < 1e-12, worst
