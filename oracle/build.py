"""Builds the FP64 CPU oracle (test infrastructure) into oracle/liborc.so.

Plain C11 with libm and pthreads, -O2, no fast-math and no SIMD intrinsics,
no fused multiply-adds; a second build fuses them (a rounding perturbation).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["oracle_core.c", "oracle_grid.c", "oracle_transport.c"]
LIB = os.path.join(HERE, "liborc.so")
# The same sources with multiply-adds fused wherever the compiler can (x86
# FMA3): identical arithmetic up to rounding.  Tests use it to measure how far
# a workload's histories move under last-bit rounding changes alone.
LIB_FMA = os.path.join(HERE, "liborc_fma.so")


def _compile(out, extra, verbose):
    cmd = ["gcc", "-std=c11", "-O2", "-fno-fast-math", "-fPIC", "-shared", "-pthread",
           "-Wall", "-Wextra", "-Wno-unused-parameter", *extra, "-o", out + ".tmp"]
    cmd += [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)


def build(verbose=False):
    _compile(LIB, ["-ffp-contract=off"], verbose)
    _compile(LIB_FMA, ["-mfma", "-ffp-contract=fast"], verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
