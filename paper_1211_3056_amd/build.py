"""Compile libhrsearch.so for gfx950 with hipcc (in-tree), and the host
library libhrcpu.so (the multi-core SIMD CPU search, for comparisons)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = [os.path.join(HERE, "csrc", "hr_lib.hip")]
OUT = os.path.join(HERE, "libhrsearch.so")
CPU_SOURCES = [os.path.join(HERE, "csrc", "cpu_search.cpp")]
CPU_OUT = os.path.join(HERE, "libhrcpu.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def _compile(cmd, out, verbose):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    if verbose:
        sys.stderr.write(r.stderr)
    os.replace(out + ".tmp", out)


def build(verbose: bool = False) -> str:
    _compile(["hipcc", *FLAGS, "-o", OUT + ".tmp", *SOURCES], OUT, verbose)
    # host code only (hr_core.h compiled for the CPU, AVX-512 chosen at run time)
    _compile(["hipcc", "-O3", "-std=c++17", "-fPIC", "-shared", "-I" + os.path.join(ROOT, "include"),
              "-o", CPU_OUT + ".tmp", *CPU_SOURCES, "-lpthread"], CPU_OUT, verbose)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
