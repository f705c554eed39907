"""Build libmindist.so (HIP kernels for gfx950 + host scheduler + C ABI).

    python -m paper_1603_06757_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmindist.so")

SOURCES = ["mindist_kernels.hip", "mindist_batch.hip", "mindist_walk.hip", "mindist_plan.cpp", "mindist_host.cpp",
           "mindist_pool.cpp", "mindist_batch.cpp", "mindist_server.cpp"]

# Packed FP32 instructions are disabled for every HIP translation unit.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIP_FLAGS, "-shared", "-I", os.path.join(ROOT, "include"), *srcs,
           "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libmindist.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
