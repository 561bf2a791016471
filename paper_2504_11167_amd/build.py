"""Build the HIP library liblrspike.so for gfx950 (in-tree, next to this file)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblrspike.so")
SOURCES = ["api.hip"]
DEPS = ["api.hip", "batched.hip", "common.h", "layout.h", "sweep.h", "factor.hip", "factor_wave.hip", "factor_lds.hip", "solve.hip",
        "solve_wave.hip", "reduced.hip", "krylov.hip", "rsvd.hip", "iter.hip", "sweep64.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def build(force: bool = True, verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    newest = max(os.path.getmtime(os.path.join(CSRC, d)) for d in DEPS)
    newest = max(newest, os.path.getmtime(os.path.join(HERE, "..", "include", "lrspike.h")))
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= newest:
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
