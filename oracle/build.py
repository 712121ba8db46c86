"""Compile the plain-C oracle into oracle/libjfft_oracle.so (gcc, -O2, OpenMP).

No -ffast-math: the oracle keeps IEEE evaluation order."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "jfft_oracle.c")
LIB = os.path.join(HERE, "libjfft_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-Wall",
           "-Wno-unknown-pragmas", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
