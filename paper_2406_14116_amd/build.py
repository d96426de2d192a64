"""Build libvbw.so (gfx950 HIP kernels + host plan code + C ABI) in-tree."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvbw.so")
SOURCES = ["ols_fft.hip", "ols_gemm.hip", "copy.hip", "stream.hip", "scratch.hip", "vbw_api.cpp"]
ARCH = os.environ.get("VBW_OFFLOAD_ARCH", "gfx950")

HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")

FLAGS = [
    "-O3", "-std=c++20", "-fPIC", f"--offload-arch={ARCH}",
    # packed float32 arithmetic stays off: plain VALU float32 only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
# per-source flags: the matrix-core kernel keeps its MFMA accumulators in
# ordinary VGPRs (no accumulator-register reads after every product)
SOURCE_FLAGS = {"ols_gemm.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def build(verbose: bool = False, extra=()) -> str:
    from concurrent.futures import ThreadPoolExecutor
    objs, cmds = [], []
    for src in SOURCES:
        obj = os.path.join(CSRC, src + ".o")
        cmds.append([HIPCC, *FLAGS, *SOURCE_FLAGS.get(src, []), *extra, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                     "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)

    def compile_one(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    # the sources are independent: compile them side by side
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as pool:
        for f in [pool.submit(compile_one, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    rocm_lib = os.path.join(os.path.dirname(os.path.dirname(HIPCC)), "lib")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-L", rocm_lib,
           "-Wl,-rpath," + rocm_lib, "-lrocprofiler-sdk-roctx", "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
