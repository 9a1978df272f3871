"""Compile the FP64 oracle (plain C + OpenMP) into oracle/liboracle.so.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
baseline load the result.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pulsar_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# IEEE double throughout: no fast-math, no FMA contraction, generic x86-64 so
# the same binary runs on any host it is copied to.
CFLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
          "-ffp-contract=off", "-march=x86-64-v2", "-Wall", "-Wextra"]


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
