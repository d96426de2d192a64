"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the C ABI's plan logic (VBW_HOST_ONLY plans, with the GPU launchers stubbed)
and the oracle's C entry points, built with g++/gcc and run; any memory or
undefined-behaviour error aborts the program."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, exe):
    subprocess.run(cmd, check=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    return r.stdout


def test_host_plan_logic_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    lib = os.path.join(ROCM, "lib")
    if gxx is None or not os.path.exists(os.path.join(lib, "libamdhip64.so")):
        pytest.skip("g++ or the HIP runtime library missing")
    exe = str(tmp_path / "host_plan_check")
    out = _run([gxx, "-std=c++20", *SAN, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
                "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2406_14116_amd", "csrc"),
                os.path.join(ROOT, "tests", "sanitize", "host_plan_check.cpp"),
                os.path.join(ROOT, "paper_2406_14116_amd", "csrc", "vbw_api.cpp"),
                "-L", lib, "-Wl,-rpath," + lib, "-lamdhip64", "-lrocprofiler-sdk-roctx", "-o", exe], exe)
    assert "0 failures" in out


def test_oracle_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc missing")
    exe = str(tmp_path / "oracle_check")
    out = _run([gcc, "-std=c11", *SAN, "-fopenmp", os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"),
                os.path.join(ROOT, "oracle", "ols_oracle.c"), "-lm", "-o", exe], exe)
    assert "ok" in out
