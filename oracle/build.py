"""Builds the oracle's shared library (plain C, FP64, OpenMP) with gcc.

Test infrastructure only: the oracle checks the GPU library and is never
part of it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["lattice.c", "moment_lb.c", "population_lb.c", "color_gradient.c", "adjoint.c", "adjoint_cg.c"]
LIB = os.path.join(HERE, "liboracle.so")
COMPILER = "gcc"
FLAGS = ["-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    cmd = [COMPILER, *FLAGS, "-o", LIB + ".tmp", *srcs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
