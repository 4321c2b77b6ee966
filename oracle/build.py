"""Build the CPU oracle (plain C, gcc, OpenMP) into ``oracle/liboracle.so``.

The oracle is test infrastructure; building it is part of the project's build
step so that the checker exists wherever the library is built.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "qaia_oracle.c")]

# Portable optimisation level: the library built here also runs on other
# x86-64 hosts, so no -march=native; x86-64-v3 (AVX2/FMA) is universal on
# current servers.  No fast-math: the oracle's float64 arithmetic is IEEE.
CFLAGS = ["-O3", "-march=x86-64-v3", "-fno-fast-math", "-ffp-contract=off",
          "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, *SOURCES, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
