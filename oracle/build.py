"""Compile the CPU oracle (test infrastructure) into oracle/liboracle.so with gcc.

Flags: -O2, -ffp-contract=off (no fused multiply-add except explicit fmaf), -mfma so that fmaf
is the hardware fused operation, no -ffast-math.  Run: python oracle/build.py
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["raster.c", "brute.c", "resolve.c", "compress.c", "texture.c"]
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra",
           "-Wno-unused-parameter", "-ffp-contract=off", "-fno-fast-math", "-mfma", "-msse4.1",
           "-o", LIB + ".tmp"] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
