"""Build the FP64 oracle shared library (test infrastructure) with gcc.

The oracle is plain C; it is compiled without fast-math so that every
operation is IEEE double precision as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ols_oracle.c")
LIB = os.path.join(HERE, "libols_oracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fno-fast-math", "-ffp-contract=off",
           "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
