"""Build libsf.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SO = os.path.join(PKG, "libsf.so")
MICRO_SO = os.path.join(PKG, "libsf_micro.so")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # keep the compiler away from packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _hipcc(src: str, out: str, verbose: bool):
    tmp = out + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           "-o", tmp, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compile libsf.so (the sketch) and libsf_micro.so (measurement kernels)."""
    _hipcc(os.path.join(PKG, "csrc", "sf_lib.hip"), SO, verbose)
    _hipcc(os.path.join(PKG, "csrc", "sf_micro.hip"), MICRO_SO, verbose)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
