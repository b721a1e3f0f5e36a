"""Build libsdfcollide.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_2110_01614_amd.build [--verbose]
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsdfcollide.so")
SOURCES = ["sdf_api.cpp", "sdf_k16.hip", "sdf_k32.hip", "sdf_train.hip", "sdf_step.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-inline-asm", "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False, extra=None) -> str:
    """Compile every source (always; a fresh build each call) and return the library path."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + list(extra or [])
    for s in SOURCES:
        if s.endswith(".cpp"):
            cmd += ["-x", "hip", os.path.join(CSRC, s)]
        else:
            cmd += ["-x", "hip", os.path.join(CSRC, s)]
    cmd += ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv))
