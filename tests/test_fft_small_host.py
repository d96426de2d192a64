"""The GPU kernels' radix-2/4/8/16 butterflies (csrc/fft_small.h), built for
the host with g++ and checked against a float64 DFT (eq. (4) sign convention):
a wrong sign, twiddle or output order gives an O(1) error, float32 rounding
about 1e-7."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2406_14116_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.isdir(os.path.join(ROCM, "include", "hip")):
        pytest.skip("g++ or HIP headers missing")
    exe = str(tmp_path_factory.mktemp("fft_small") / "check")
    subprocess.run([gxx, "-O1", "-std=c++20", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
                    "-I", CSRC, os.path.join(os.path.dirname(__file__), "fft_small_check.cpp"), "-o", exe],
                   check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    res = {}
    for line in out.split("\n"):
        if line.strip():
            r, inv, err = line.split()
            res[(int(r), int(inv))] = float(err)
    return res


@pytest.mark.parametrize("r", [2, 4, 8, 16])
@pytest.mark.parametrize("inv", [0, 1])
def test_butterfly_matches_dft(results, r, inv):
    assert results[(r, inv)] < 3e-7, results
