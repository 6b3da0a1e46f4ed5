"""Build libjso.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2309_15676_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libjso.so")
SOURCES = ["kernels.hip", "api.hip", "bvh.cpp", "ubench.hip"]
ARCH = os.environ.get("JSO_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    # contract only within one source expression: the forward pass and the
    # replay must round every radiance term identically
    "-ffp-contract=on",
    # no packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FP32 division and square root by the hardware reciprocal / square-root
    # instructions (about 1 ulp) instead of the correctly rounded sequences;
    # far inside the FP32-vs-FP64 tolerance, 15% fewer instructions per vertex
    "-fno-hip-fp32-correctly-rounded-divide-sqrt",
    "-I" + os.path.join(ROOT, "include"),
    "-I" + CSRC,
]


def build(verbose: bool = False) -> str:
    """Compile every source and link libjso.so; always rebuilds."""
    from concurrent.futures import ThreadPoolExecutor
    hipcc = os.environ.get("HIPCC", "hipcc")
    objs = [os.path.join(CSRC, os.path.splitext(src)[0] + ".o") for src in SOURCES]

    def compile_one(k):
        cmd = [hipcc, *FLAGS, "-c", os.path.join(CSRC, SOURCES[k]), "-o", objs[k]]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True, stderr=None if verbose else subprocess.PIPE)

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as pool:
        list(pool.map(compile_one, range(len(SOURCES))))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
