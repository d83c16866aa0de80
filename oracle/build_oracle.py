"""Compile the FP64 gemm reference (gemm_ref.c) into liboracle.so with gcc.

Test infrastructure only: the library it builds is loaded by the tests, the
smoke check and the CPU-baseline leg of the benchmark.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gemm_ref.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    """Always recompiles; returns the path of the shared library."""
    # -O2 without -march: the x86-64 baseline has no FMA, so every product and
    # sum is rounded separately, exactly as written in the C source.
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", SRC, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
