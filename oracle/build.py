"""Build the C oracle into oracle/_liboracle.so with gcc.

Test infrastructure only: the product library never links or loads it.
Flags: -O2, hardware fma for fmaf, no floating-point contraction and no
fast-math, so every binary32 operation in the oracle's step is the one
written in the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fpt_oracle.c")
LIB = os.path.join(HERE, "_liboracle.so")

CFLAGS = ["-O2", "-mfma", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11",
          "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", *CFLAGS, SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
