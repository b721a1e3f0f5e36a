"""Build libsdfcollide.so (HIP for gfx950) in-tree with hipcc.

Every translation unit is compiled to an object in parallel (the 16-bit
kernel file once per hidden width and operand type), then the objects are linked into the
shared library.

Usage: python -m paper_2110_01614_amd.build [--verbose] [-jN]
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsdfcollide.so")
OBJDIR = os.path.join(os.path.dirname(HERE), "_build", "obj")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# (source, extra defines, object name)
# 16-bit kernel instantiations: (hidden width, operand type: 1 BF16, 2 FP16,
# 3 BF16x3, 4 FP8); FP8 exists from width 128; the persistent grouped kernel
# (all widths 128-512 in one kernel) per operand type
K16_UNITS = [(w, p) for w in (64, 128, 256, 512) for p in (1, 2, 3, 4) if not (w == 64 and p == 4)]
UNITS = [("sdf_k16.hip", ["-DSDF_K16_WIDTH=%d" % w, "-DSDF_K16_PREC=%d" % p], "sdf_k16_w%d_p%d" % (w, p))
         for w, p in sorted(K16_UNITS, key=lambda u: -u[0])] + \
        [("sdf_k16.hip", ["-DSDF_K16_PERSIST", "-DSDF_K16_WIDTH=0", "-DSDF_K16_PREC=%d" % p], "sdf_k16_persist_p%d" % p)
         for p in (1, 2, 3, 4)] + \
        [(s, [], os.path.splitext(s)[0]) for s in ("sdf_api.cpp", "sdf_k32.hip", "sdf_train.hip", "sdf_step.hip")]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-inline-asm", "-Wno-unused-command-line-argument",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)  # the host pass does not know the feature
    if r.returncode != 0:
        raise RuntimeError("hipcc failed (%d):\n%s\n%s" % (r.returncode, " ".join(cmd), msg))
    if msg.strip() and verbose:
        print(msg, flush=True)


def build(verbose: bool = False, extra=None, jobs: int | None = None) -> str:
    """Compile every source (always; a fresh build each call) and return the library path."""
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(16, len(UNITS), os.cpu_count() or 1)
    cmds, objs = [], []
    for src, defs, name in UNITS:
        obj = os.path.join(OBJDIR, name + ".o")
        objs.append(obj)
        cmds.append([HIPCC] + FLAGS + list(extra or []) + defs +
                    ["-c", "-x", "hip", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    j = [int(a[2:]) for a in sys.argv[1:] if a.startswith("-j")]
    print(build(verbose="--verbose" in sys.argv, jobs=j[0] if j else None))
