"""Builds the FP64 CPU oracle (test infrastructure) into oracle/liborc.so.

Plain C11 with libm and pthreads, -O2, no fast-math and no SIMD intrinsics.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["oracle_core.c", "oracle_grid.c", "oracle_transport.c"]
LIB = os.path.join(HERE, "liborc.so")


def build(verbose=False):
    cmd = ["gcc", "-std=c11", "-O2", "-fno-fast-math", "-fPIC", "-shared", "-pthread",
           "-Wall", "-Wextra", "-Wno-unused-parameter", "-o", LIB + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
