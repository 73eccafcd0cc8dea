"""Build libmanta.so for gfx950 with hipcc (in-tree).

Floating point flags are part of the step contract: no contraction of a*b+c
into FMA, IEEE-correct binary32 division and square root, no flushing of
denormals, and no packed-FP32 instructions.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "manta.hip")
DEPS = [SRC, os.path.join(HERE, "csrc", "step_kernels.hpp"), os.path.join(HERE, "csrc", "device_math.hpp"),
        os.path.join(HERE, "csrc", "routing.hpp"), os.path.join(ROOT, "include", "manta.h")]
LIB = os.path.join(HERE, "libmanta.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt", "-fno-gpu-flush-denormals-to-zero",
    "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile (always, when force) and return the library path."""
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(p) for p in DEPS):
        return LIB
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
