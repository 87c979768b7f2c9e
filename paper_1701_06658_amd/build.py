"""Build the HIP library (gfx950) in-tree: ``python -m paper_1701_06658_amd.build``."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "gg_lib.hip")
DEPS = [SRC, os.path.join(HERE, "csrc", "gg_kernels.hpp"), os.path.join(HERE, "csrc", "gg_march.hpp"),
        os.path.join(HERE, "csrc", "gg_closest.hpp"),
        os.path.join(ROOT, "include", "gg.h")]
LIB = os.path.join(HERE, "libgg.so")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # FP64 path: no contraction, products and sums rounded separately (FP32 uses explicit FMA)
    "-ffp-contract=off",
    # packed FP32 instructions stay off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # device code: no NaN ever occurs on the path, so min / max need no quieting
    "-Xarch_device", "-fno-honor-nans",
    "-Wall", "-Wno-unused-result",
]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build_library(verbose=False):
    """Compile libgg.so for gfx950 (always recompiles)."""
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build_library(verbose="-v" in sys.argv)
    print(LIB)
