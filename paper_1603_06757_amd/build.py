"""Build libmindist.so (HIP kernels for gfx950 + host scheduler + C ABI)
and libmindist_cpu.so (the paper's CPU algorithms as host baselines, plain C
with OpenMP; the GPU library does not link or call it).

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
CPU_LIB = os.path.join(HERE, "libmindist_cpu.so")
# x86-64 with POPCNT: the library runs on whichever host drives the GPU
CPU_FLAGS = ["-O3", "-fPIC", "-shared", "-fopenmp", "-mpopcnt", "-std=c11"]

SOURCES = ["mindist_kernels.hip", "mindist_batch.hip", "mindist_walk.hip", "mindist_plan.cpp", "mindist_host.cpp",
           "mindist_pool.cpp", "mindist_batch.cpp", "mindist_server.cpp", "mindist_noalloc.hip"]

# Packed FP32 instructions are disabled for every HIP translation unit.
# Matrix-core results go to VGPRs, where the minima read them, instead of
# AGPRs (which would add one v_accvgpr_read per result).
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-mllvm", "-amdgpu-mfma-vgpr-form",
             "-Wno-unused-command-line-argument"]


def _compile(hipcc: str, src: str, obj: str, verbose: bool) -> None:
    cmd = [hipcc, *HIP_FLAGS, "-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed compiling {os.path.basename(src)}")


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source (in parallel, one object each, under a private
    build folder) and link libmindist.so; then the CPU baseline library."""
    from concurrent.futures import ThreadPoolExecutor

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs = [os.path.join(objdir, os.path.basename(s) + ".o") for s in srcs]
    jobs = jobs or min(len(srcs), max(1, min(os.cpu_count() or 1, 8)))
    with ThreadPoolExecutor(jobs) as ex:
        list(ex.map(lambda so: _compile(hipcc, so[0], so[1], verbose), zip(srcs, objs)))
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIP_FLAGS, "-shared", *objs, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed linking libmindist.so")
    os.replace(tmp, LIB)
    build_cpu(verbose)
    return LIB


def build_cpu(verbose: bool = False) -> str:
    tmp = CPU_LIB + ".tmp"
    cmd = ["gcc", *CPU_FLAGS, "-I", os.path.join(ROOT, "include"),
           os.path.join(CSRC, "mindist_cpu.c"), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("gcc failed building libmindist_cpu.so")
    os.replace(tmp, CPU_LIB)
    return CPU_LIB


if __name__ == "__main__":
    print(build(verbose=True))
