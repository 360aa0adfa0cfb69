"""Build libsf.so (the sketch library) and libsf_micro.so (measurement
kernels) in-tree with hipcc for gfx950.  Translation units compile in
parallel, then link."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SO = os.path.join(PKG, "libsf.so")
MICRO_SO = os.path.join(PKG, "libsf_micro.so")
OBJ = os.path.join(PKG, "_build")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # keep the compiler away from packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]
INCLUDES = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]

LIBS = {
    SO: ["sf_lib.hip", "sf_group.hip", "sf_pool.hip"],
    MICRO_SO: ["sf_micro.hip"],
}


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False) -> str:
    """Compile every translation unit (always), then link both libraries."""
    os.makedirs(OBJ, exist_ok=True)
    jobs = []
    for so, srcs in LIBS.items():
        for src in srcs:
            obj = os.path.join(OBJ, src.replace(".hip", ".o"))
            jobs.append(["hipcc", *HIPCC_FLAGS, *INCLUDES, "-c", "-o", obj,
                         os.path.join(PKG, "csrc", src)])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for f in [ex.submit(_run, j, verbose) for j in jobs]:
            f.result()
    for so, srcs in LIBS.items():
        tmp = so + ".tmp"
        objs = [os.path.join(OBJ, s.replace(".hip", ".o")) for s in srcs]
        _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
        os.replace(tmp, so)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
