"""Builds the oracle's C part (test infrastructure only) with gcc.

liboracle.so: the sequential oracle, -O2 -ffp-contract=off: every multiply
and add separately rounded, in the order the source writes them.
liboracle_omp.so: the all-cores build of the same CG (OpenMP), for the CPU
baseline of the benchmark and its floor solutions; -O3 for x86-64-v3
(AVX2-class hosts), contraction off as well.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ss_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
SRC_OMP = os.path.join(HERE, "ss_oracle_omp.c")
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")

COMMON = ["-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra"]


def _gcc(flags, src, lib, verbose):
    cmd = ["gcc", *flags, *COMMON, "-o", lib + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)


def build(verbose: bool = False) -> str:
    _gcc(["-O2"], SRC, LIB, verbose)
    _gcc(["-O3", "-march=x86-64-v3", "-fopenmp"], SRC_OMP, LIB_OMP, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
