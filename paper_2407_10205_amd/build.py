"""Build libphia.so (HIP kernels + host runtime + C ABI) for gfx950 with hipcc.

Every source is compiled to an object of its own (in parallel, under
_build/), then the objects are linked into the shared library.  Each HIP
kernel is launched from the file that defines it, so no relocatable device
code is needed.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libphia.so")
OBJDIR = os.path.join(PKG, "_build")

SOURCES = ["phia_kernels.hip", "phia_batch_kernel.hip", "phia_valu_kernel.hip", "phia_runtime.cpp", "phia_batch.cpp",
           "phia_server.cpp", "phia_server_kernels.hip", "phia_noalloc.hip"]

# -ffp-contract=off: no implicit fused multiply-adds (the sweep's op sequence
# is fixed and every fma is explicit).  Correctly rounded FP32 division and
# square root (HIP's default, stated).  Packed FP32 instructions disabled.
HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _compile(src, verbose):
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *HIPFLAGS, "-I", INCLUDE, "-I", CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def build(verbose=False, jobs=None):
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    out = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
