"""Build libpxt.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2104_06573_amd.build

The library is csrc/pxt.hip (kernels and the C ABI) and csrc/server.cpp
(the continuous-batching server over that ABI), built
for gfx950 only, without floating-point contraction (the double-precision
cuts must round exactly as written) and with packed FP32 instructions
disabled.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", "pxt.hip"), os.path.join(HERE, "csrc", "server.cpp")]
LIB = os.path.join(HERE, "libpxt.so")
ARCH = "gfx950"

FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose=False, extra=()):
    """Compile csrc/ into libpxt.so next to this file; returns its path."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + FLAGS + list(extra) + [
        "-I", os.path.join(ROOT, "include"),
        "-I", os.path.join(HERE, "csrc"),
        "-o", tmp,
    ] + SRCS + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
