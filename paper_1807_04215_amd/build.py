"""Build libgridspt.so for gfx950 with hipcc (in-tree, next to this file).

The library is one translation unit for the C ABI (csrc/gridspt.hip) plus one
per grid size (csrc/sizes/n*.hip); they compile in parallel into _build/ and
link into libgridspt.so.
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgridspt.so")

ARCH = "--offload-arch=gfx950"
HIPCC_FLAGS = [
    ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions stay off: some of their forms have given wrong results
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def sources() -> list[str]:
    return [os.path.join(CSRC, "gridspt.hip")] + sorted(glob.glob(os.path.join(CSRC, "sizes", "n*.hip")))


def _compile(hipcc: str, src: str, verbose: bool) -> str:
    rel = os.path.relpath(src, CSRC).replace(os.sep, "_")
    obj = os.path.join(OBJDIR, os.path.splitext(rel)[0] + ".o")
    cmd = [hipcc, *HIPCC_FLAGS, "-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or max(1, min(8, os.cpu_count() or 1))
    srcs = sources()
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(hipcc, s, verbose), srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, ARCH, "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
