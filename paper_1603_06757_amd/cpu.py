"""ctypes binding of libmindist_cpu.so: the paper's CPU enumeration
algorithms (Section 3) for one pair, as measured host baselines.  Not used by
the GPU path."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmindist_cpu.so")
ALGORITHMS = {"basic": 0, "optimized": 1, "stack": 2, "saved": 3, "saved_unroll2": 4}
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1603_06757_amd.build`")
        L = C.CDLL(LIB_PATH)
        u64p = C.POINTER(C.c_uint64)
        L.mindist_cpu_pair.argtypes = [u64p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                       C.c_int, C.POINTER(C.c_int32), u64p, u64p,
                                       C.POINTER(C.c_double)]
        _lib = L
    return _lib


def cpu_pair(rows, k: int, w: int, algorithm: str, s: int = 5, threads: int = 0,
             offset: int = 0) -> dict:
    """Pair (rows, w): rows is (k, words) uint64; weight = offset + popcount."""
    R = np.ascontiguousarray(rows, dtype=np.uint64)
    if R.ndim != 2 or R.shape[0] != k:
        raise ValueError("rows must be (k, words)")
    pm, cb, ad, ts = C.c_int32(), C.c_uint64(), C.c_uint64(), C.c_double()
    rc = lib().mindist_cpu_pair(R.ctypes.data_as(C.POINTER(C.c_uint64)), k, R.shape[1], w, offset,
                                ALGORITHMS[algorithm], s, threads, C.byref(pm), C.byref(cb),
                                C.byref(ad), C.byref(ts))
    if rc:
        raise RuntimeError(f"mindist_cpu_pair failed ({rc})")
    return {"pair_min": pm.value, "combinations": cb.value, "additions": ad.value,
            "table_seconds": ts.value}
