"""Compile the C oracle into oracle/liboracle.so with gcc (test infrastructure).

The in-tree library targets x86-64-v3 (AVX2 and FMA), so that one build
runs on every host the tests may use.  ``build(native=True, out=...)``
compiles a copy for the CPU it runs on (``-march=native``); the benchmark's
CPU-baseline leg times that copy on the host where it runs.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "phia_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# -ffp-contract=off: no implicit fused multiply-adds; every fmaf is explicit.
# -fno-fast-math keeps IEEE semantics (no reassociation), so vectorised FP32
# loops give the same bits as scalar ones.
CFLAGS = ["-O3", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
          "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(verbose=False, native=False, out=None):
    out = out or LIB
    arch = "-march=native" if native else "-march=x86-64-v3"
    cmd = ["gcc", *CFLAGS, arch, SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, native="--native" in sys.argv)
