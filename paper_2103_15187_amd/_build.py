"""Build libfsei.so (HIP kernels for gfx950 + host plan code) in-tree."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libfsei.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["fsei_api.hip", "fsei_plan.cpp"]
HEADERS = ["fsei_plan.h", "fsei_fft.h", "fsei_transforms.h", "fsei_kernels.h", "fsei_viscous.h",
           "fsei_momentum.h", "fsei_ibm.h"]

# -packed-fp32-ops: hipcc -O3 may otherwise emit packed FP32 instructions
# from ordinary float code; this keeps them out of every kernel.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def build(verbose: bool = True) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(PKG, "..", "include"), *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
