"""Compile the oracle's C++ sources into oracle/liboracle.so (g++, FP64,
no FMA contraction, OpenMP over independent cells)."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SOURCES = ["oracle_capi.cpp", "amr_oracle.cpp", "adjoint_oracle.cpp"]
HEADERS = ["scheme.hpp"]


def build(verbose=False):
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    # -O3 and the x86-64-v3 level (AVX2; every host this runs on has it): the
    # vectoriser does not reassociate without -ffast-math and contraction is
    # off, so the arithmetic is that of the plain -O2 build
    cmd = ["g++", "-O3", "-march=x86-64-v3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared",
           "-Wall", "-Wno-unknown-pragmas", "-o", LIB + ".tmp"] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=HERE)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def needs_build():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(os.path.join(HERE, f)) > t for f in SOURCES + HEADERS)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
