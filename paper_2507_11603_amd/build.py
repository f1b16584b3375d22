"""Build libthor.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", f) for f in ("thor_lib.hip", "thor_rays.hip")]
LIB = os.path.join(HERE, "libthor.so")
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("thor_device.hpp", "thor_engine.hpp")] + \
          [os.path.join(ROOT, "include", f) for f in ("thor.h", "thor_rays.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-munsafe-fp-atomics",
    # multiply-adds fused only within one expression: every kernel that
    # evaluates the same formula rounds it the same way
    "-ffp-contract=on",
    # packed FP32 instructions are disabled on this target on purpose
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in SRCS + HEADERS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc"] + HIPCC_FLAGS + ["-o", tmp] + SRCS
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose=True)
    print(LIB)
    sys.exit(0)
