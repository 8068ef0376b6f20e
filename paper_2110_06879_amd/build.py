"""Build the gfx950 HIP library ``libacopf.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB_DIR = os.path.join(HERE, "_lib")
LIB_PATH = os.path.join(LIB_DIR, "libacopf.so")
SOURCES = ["acopf.hip", "branch_kernel.hip", "server.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no implicit contraction: the iteration reproduces a fixed IEEE
    # operation sequence, with fused multiply-adds only where written out
    "-ffp-contract=off",
    # no packed FP32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # LLVM's iterative ILP-oriented machine scheduler: the branch kernel runs
    # at one wavefront per SIMD, where instruction-level parallelism within
    # a lane is what hides latency (3% faster x-step on the 70k grid; the
    # operations and their order are unchanged)
    "-mllvm", "-amdgpu-sched-strategy=iterative-ilp",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def build(verbose: bool = True, extra: list[str] | None = None) -> str:
    """Compile every HIP source of the library for gfx950 (always rebuilds)."""
    os.makedirs(LIB_DIR, exist_ok=True)
    tmp = LIB_PATH + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *(extra or []), "-I", os.path.join(ROOT, "include"),
           "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    out = subprocess.run(cmd, capture_output=True, text=True)
    if out.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out.stdout + out.stderr)
    if verbose and out.stderr.strip():
        print(out.stderr, file=sys.stderr)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    build()
