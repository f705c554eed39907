"""ctypes wrapper of the CPU oracle (mindist_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mindist_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORC_MAXG = 64


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, pthreads)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared",
                               "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        u64p = C.POINTER(C.c_uint64)
        ip = C.POINTER(C.c_int)
        L.orc_binom.restype = C.c_uint64
        L.orc_binom.argtypes = [C.c_int, C.c_int]
        L.orc_brute.restype = C.c_int
        L.orc_brute.argtypes = [u64p, C.c_int, C.c_int, u64p, u64p]
        L.orc_partition.restype = C.c_int
        L.orc_partition.argtypes = [u64p, C.c_int, C.c_int, ip, ip, ip]
        L.orc_gamma.restype = C.c_int
        L.orc_gamma.argtypes = [u64p, C.c_int, C.c_int, ip, C.c_int, u64p]
        L.orc_pair.restype = C.c_int
        L.orc_pair.argtypes = [u64p, C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_uint64,
                               C.c_int, u64p, u64p, u64p, u64p]
        L.orc_combo_codeword.restype = C.c_int
        L.orc_combo_codeword.argtypes = [u64p, C.c_int, C.c_int, C.c_int, C.c_uint64, ip, u64p]
        L.orc_set_fault.restype = None
        L.orc_set_fault.argtypes = [C.c_int]
        L.orc_bz.restype = C.c_int
        L.orc_bz.argtypes = [u64p, C.c_int, C.c_int, C.c_void_p, C.c_int,
                             ip, u64p, ip, u64p, ip, C.c_int, ip, u64p, ip, u64p]
        _lib = L
    return _lib


class _Opts(C.Structure):
    _fields_ = [("term_per_level", C.c_int), ("partial_policy", C.c_int), ("threads", C.c_int)]


def _u64(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def _i32(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _mat(G):
    G = np.ascontiguousarray(G, dtype=np.uint64)
    return G


class OracleError(RuntimeError):
    pass


def _check(rc):
    if rc < 0:
        raise OracleError({-1: "E_ARG", -2: "E_RANK", -4: "E_NOMEM", -6: "E_LIMIT"}.get(rc, rc))
    return rc


class planted:
    """Context manager for the tests that show the pins catch mistakes:
    plants mistake `fault` (see the list in mindist_oracle.c) in the oracle
    for the duration of the block."""

    def __init__(self, fault: int):
        self.fault = fault

    def __enter__(self):
        lib().orc_set_fault(self.fault)
        return self

    def __exit__(self, *exc):
        lib().orc_set_fault(0)


def binom(n: int, r: int) -> int:
    return int(lib().orc_binom(n, r))


def brute(G, n: int, k: int):
    """Plain definition: (d, weight distribution A_0..A_n, witness words)."""
    G = _mat(G)
    W = (n + 63) // 64
    dist = np.zeros(n + 1, dtype=np.uint64)
    wit = np.zeros(W, dtype=np.uint64)
    d = _check(lib().orc_brute(_u64(G), n, k, _u64(dist), _u64(wit)))
    return d, dist, wit


def partition(G, n: int, k: int):
    """Greedy disjoint information sets: (list of full sets, partial set)."""
    G = _mat(G)
    sets = np.zeros(n, dtype=np.int32)
    mf, km = C.c_int(0), C.c_int(0)
    _check(lib().orc_partition(_u64(G), n, k, _i32(sets), C.byref(mf), C.byref(km)))
    full = [sets[j * k:(j + 1) * k].tolist() for j in range(mf.value)]
    part = sets[mf.value * k: mf.value * k + km.value].tolist()
    return full, part


def gamma(G, n: int, k: int, first):
    """RREF of G under column order (first ascending, then the rest)."""
    G = _mat(G)
    W = (n + 63) // 64
    f = np.ascontiguousarray(first, dtype=np.int32)
    out = np.zeros((k, W), dtype=np.uint64)
    _check(lib().orc_gamma(_u64(G), n, k, _i32(f), len(f), _u64(out)))
    return out


def pair(Gam, n: int, k: int, g: int, lo: int = 0, hi: int = (1 << 64) - 1, threads: int = 1):
    """(min weight, lex rank of first min, weight sum, count, row additions)."""
    Gam = _mat(Gam)
    mr, ws, cnt, adds = C.c_uint64(0), C.c_uint64(0), C.c_uint64(0), C.c_uint64(0)
    m = _check(lib().orc_pair(_u64(Gam), n, k, g, lo, hi, threads,
                              C.byref(mr), C.byref(ws), C.byref(cnt), C.byref(adds)))
    return m, mr.value, ws.value, cnt.value, adds.value


def combo_codeword(Gam, n: int, k: int, g: int, rank: int):
    Gam = _mat(Gam)
    W = (n + 63) // 64
    combo = np.zeros(g, dtype=np.int32)
    word = np.zeros(W, dtype=np.uint64)
    _check(lib().orc_combo_codeword(_u64(Gam), n, k, g, rank, _i32(combo), _u64(word)))
    return combo.tolist(), word


PARTIAL_POLICIES = {"always": 0, "never": 1, "when_useful": 2}


def bz(G, n: int, k: int, per_level: bool = False, partial_never: bool = False,
       threads: int = 1, partial: str | None = None) -> dict:
    """Algorithm 1 (Brouwer-Zimmerman) under the canonical readings.
    partial: "always" (default), "never" (same as partial_never=True) or
    "when_useful" (the partial set from the first level its bound term is
    positive, with its lower levels caught up then)."""
    policy = PARTIAL_POLICIES[partial] if partial else (1 if partial_never else 0)
    G = _mat(G)
    W = (n + 63) // 64
    cap = n + 1
    sets = np.zeros(n, dtype=np.int32)
    counts = np.zeros(cap * (k + 1), dtype=np.uint64)
    pmin = np.zeros(cap * (k + 1), dtype=np.int32)
    wsum = np.zeros(cap * (k + 1), dtype=np.uint64)
    tcap = 4096
    trace = np.zeros(6 * tcap, dtype=np.int32)
    info = np.zeros(8, dtype=np.int32)
    wit = np.zeros(W, dtype=np.uint64)
    wcombo = np.zeros(ORC_MAXG, dtype=np.int32)
    wmeta = np.zeros(3, dtype=np.uint64)
    opts = _Opts(1 if per_level else 0, policy, threads)
    _check(lib().orc_bz(_u64(G), n, k, C.cast(C.pointer(opts), C.c_void_p), cap,
                        _i32(sets), _u64(counts), _i32(pmin), _u64(wsum),
                        _i32(trace), tcap, _i32(info), _u64(wit), _i32(wcombo), _u64(wmeta)))
    d, m_full, k_m, ng, npairs, L, U_found, last_g = [int(x) for x in info]
    trace = trace[:6 * min(npairs, tcap)].reshape(-1, 6)
    return {
        "d": d, "m_full": m_full, "k_m": k_m, "n_gamma": ng, "pairs": npairs,
        "L_final": L, "U_found": U_found, "last_level": last_g,
        "sets": sets, "counts": counts.reshape(cap, k + 1)[:ng].copy(),
        "pair_min": pmin.reshape(cap, k + 1)[:ng].copy(),
        "wsum": wsum.reshape(cap, k + 1)[:ng].copy(),
        "trace": trace, "witness": wit,
        "witness_combo": wcombo[:int(wmeta[1])].tolist(),
        "witness_pair": (int(wmeta[0]), int(wmeta[1])), "witness_rank": int(wmeta[2]),
    }
