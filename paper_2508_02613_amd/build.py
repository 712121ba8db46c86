"""Build libjfft.so (the gfx950 HIP library behind include/jfft.h) in-tree.

hipcc cross-compiles for gfx950 without a GPU.  Packed FP32 instructions are
disabled (-packed-fp32-ops) for every device function."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libjfft.so")
SOURCES = ["jfft_api.hip"]
HEADERS = ["jfft_common.h", "stencil.h", "fft.h", "cg.h"]


def hipcc_cmd(out: str, extra=()):
    return ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            "-shared", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Werror=uninitialized", "-Werror=sometimes-uninitialized",
            "-Werror=return-type",
            "-I", os.path.join(ROOT, "include"), *extra,
            *[os.path.join(CSRC, s) for s in SOURCES], "-o", out]


def build(verbose: bool = False, extra=()) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp, extra)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
