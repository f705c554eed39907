"""Python binding of libmindist.so (the MI355X minimum-distance library).

Argument marshalling only: every step of the computation runs in the C++
host code and the HIP kernels of the library.  The binding raises if the
library has not been built; there is no fallback.

PyTorch interop (a torch stream passed as the "stream" option): torch ships
its own HIP runtime, and a process must hold only one.  If torch is imported
before this module first loads the library, the library binds to torch's
runtime and torch's streams are valid for it; if the library loads first,
passing a torch stream raises MindistError(E_ARG).
"""
from __future__ import annotations

import ctypes as C
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmindist.so")

E_NAMES = {0: "OK", -1: "E_ARG", -2: "E_RANK", -3: "E_NOMEM", -4: "E_HIP", -5: "E_LIMIT",
           -6: "E_CANCELLED", -7: "E_TIMEOUT", -8: "E_STATE", -9: "E_CERT"}

OPT = {"term": 1, "midpair_exit": 2, "partial": 3, "verify": 4, "stream": 5,
       "deadline_ms": 6, "tile_t": 7, "blocks_per_cu": 8, "profile": 9,
       "cancel_after_chunks": 10, "table_mib": 11, "lane_items": 12,
       "left_tables": 13, "chunk_order": 14, "counters": 15, "min_items": 16, "speculate": 17,
       "inject_u": 18, "mfma": 19}

MAX_WORDS = 8

# MINDIST_OPT_PARTIAL values
PARTIAL = {"always": 0, "never": 1, "when_useful": 2}


class MindistError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{E_NAMES.get(code, code)}: {msg}")
        self.code = code


class Result(C.Structure):
    _fields_ = [("d", C.c_int32), ("n", C.c_int32), ("k", C.c_int32), ("m_full", C.c_int32),
                ("k_partial", C.c_int32), ("n_gamma", C.c_int32), ("w_last", C.c_int32),
                ("j_last", C.c_int32), ("L_final", C.c_int32), ("U_found", C.c_int32),
                ("pairs_visited", C.c_int32), ("exited_midpair", C.c_int32),
                ("witness_j", C.c_int32), ("witness_w", C.c_int32),
                ("witness", C.c_uint64 * MAX_WORDS), ("witness_rows", C.c_uint64 * MAX_WORDS),
                ("executed_total", C.c_uint64), ("canonical_total", C.c_uint64),
                ("seconds_total", C.c_double), ("seconds_enum", C.c_double),
                ("enum_launches", C.c_int32), ("reserved", C.c_int32)]

    def to_dict(self):
        W = (self.n + 63) // 64
        return {
            "d": self.d, "n": self.n, "k": self.k, "m_full": self.m_full,
            "k_partial": self.k_partial, "n_gamma": self.n_gamma, "w_last": self.w_last,
            "j_last": self.j_last, "L_final": self.L_final, "U_found": self.U_found,
            "pairs_visited": self.pairs_visited, "exited_midpair": self.exited_midpair,
            "witness_pair": (self.witness_j, self.witness_w),
            "witness": np.array(self.witness[:W], dtype=np.uint64),
            "witness_rows": _set_bits(self.witness_rows, self.k),
            "executed_total": self.executed_total, "canonical_total": self.canonical_total,
            "seconds_total": self.seconds_total, "seconds_enum": self.seconds_enum,
            "enum_launches": self.enum_launches,
        }


def _set_bits(words, limit: int):
    """Indices below limit of the set bits of a little-endian uint64 word
    array, ascending (one step per set bit)."""
    out = []
    for wi in range((limit + 63) // 64):
        v = words[wi]
        while v:
            low = v & -v
            i = wi * 64 + low.bit_length() - 1
            if i >= limit:
                break
            out.append(i)
            v ^= low
    return out


class Pair(C.Structure):
    _fields_ = [("j", C.c_int32), ("w", C.c_int32), ("L_before", C.c_int32),
                ("L_after", C.c_int32), ("U_after", C.c_int32), ("pair_min", C.c_int32),
                ("count", C.c_uint64), ("executed", C.c_uint64), ("wsum", C.c_uint64),
                ("ms", C.c_double), ("dwords", C.c_int32), ("split_a", C.c_int32),
                ("split_b", C.c_int32), ("split_b2", C.c_int32), ("launch", C.c_int32),
                ("t_start_ms", C.c_double), ("dev_ms", C.c_double)]

    def to_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


# Pair records viewed as a numpy structured array (the same bytes), so that
# thousands of them become dicts without a ctypes attribute read per field
_PAIR_NAMES = [f for f, _ in Pair._fields_]
_NP_OF = {C.c_int32: np.int32, C.c_uint64: np.uint64, C.c_double: np.float64}
_PAIR_DTYPE = np.dtype({"names": _PAIR_NAMES,
                        "formats": [_NP_OF[t] for _, t in Pair._fields_],
                        "offsets": [getattr(Pair, f).offset for f in _PAIR_NAMES],
                        "itemsize": C.sizeof(Pair)})


def _pair_dicts(arr, lo: int, hi: int):
    """Records lo..hi-1 of a ctypes Pair array as dicts."""
    if hi <= lo:
        return []
    view = np.frombuffer(arr, dtype=_PAIR_DTYPE, count=hi, offset=0)[lo:hi]
    return [dict(zip(_PAIR_NAMES, t)) for t in view.tolist()]


class CertSpec(C.Structure):
    _fields_ = [("n", C.c_int32), ("k", C.c_int32), ("m_full", C.c_int32), ("k_partial", C.c_int32),
                ("partial_policy", C.c_int32), ("per_level", C.c_int32), ("midpair_exit", C.c_int32)]


class BatchOpts(C.Structure):
    _fields_ = [("tile_min", C.c_int32), ("tile_max", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("use_graph", C.c_int32), ("table_kib", C.c_int32), ("jobs_per_code", C.c_int32),
                ("chunks_per_visit", C.c_int32), ("direct_log2", C.c_int32),
                ("deadline_s", C.c_double), ("stream", C.c_int64), ("pairs", C.c_void_p), ("pairs_cap", C.c_int64),
                ("pairs_index", C.c_void_p), ("seconds_kernel", C.c_double),
                ("seconds_total", C.c_double), ("seconds_prep", C.c_double),
                ("executed_total", C.c_uint64), ("wave_s_table", C.c_double),
                ("wave_s_pair", C.c_double), ("wave_s_flush", C.c_double), ("waves", C.c_int64),
                ("chunks_table", C.c_uint64), ("chunks_pair", C.c_uint64), ("done_s", C.c_void_p)]


SERVER_MAX_PAIRS = 256


class ServerOpts(C.Structure):
    _fields_ = [("max_active", C.c_int32), ("blocks_per_cu", C.c_int32),
                ("device_bytes", C.c_int64), ("epoch_min_ms", C.c_double),
                ("table_kib", C.c_int32), ("jobs_per_code", C.c_int32),
                ("chunks_per_visit", C.c_int32), ("engine", C.c_int32), ("linger_ms", C.c_double),
                ("route_log2", C.c_int32)]


class ServerResult(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("status", C.c_int32), ("n_pairs", C.c_int32),
                ("result", Result), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_done", C.c_double), ("pairs", Pair * SERVER_MAX_PAIRS)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("admitted", C.c_uint64), ("completed", C.c_uint64),
                ("epochs", C.c_uint64), ("seconds_kernel", C.c_double),
                ("resident", C.c_int32), ("pending", C.c_int32), ("admitted_live", C.c_uint64),
                ("routed", C.c_uint64)]


_lib = None
_with_torch = False      # torch was loaded before the library (one HIP runtime)


def lib():
    """Load libmindist.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1603_06757_amd.build`")
        global _with_torch
        _with_torch = "torch" in sys.modules
        L = C.CDLL(LIB_PATH)
        u64p, ip, vp = C.POINTER(C.c_uint64), C.POINTER(C.c_int), C.c_void_p
        L.mindist_create.argtypes = [u64p, C.c_int, C.c_int, C.POINTER(vp)]
        L.mindist_set_option.argtypes = [vp, C.c_int, C.c_int64]
        L.mindist_info.argtypes = [vp, ip, ip, ip]
        L.mindist_run.argtypes = [vp, C.POINTER(Result)]
        L.mindist_get_pairs.argtypes = [vp, C.POINTER(Pair), C.c_int, ip]
        L.mindist_destroy.argtypes = [vp]
        L.mindist_destroy.restype = None
        L.mindist_last_error.restype = C.c_char_p
        L.mindist_plan.argtypes = [u64p, C.c_int, C.c_int, ip, ip, ip, u64p]
        L.mindist_bound_after.argtypes = [C.c_int] * 6
        L.mindist_colex_unrank.argtypes = [C.c_uint64, C.c_int, C.c_int, ip]
        L.mindist_run_noalloc.argtypes = [u64p, C.c_int, C.c_int, C.c_int64, C.POINTER(Result),
                                          C.POINTER(Pair), C.c_int, ip]
        L.mindist_schedule.argtypes = [C.c_int] * 5 + [C.POINTER(C.c_int32), C.c_int, ip]
        L.mindist_certify.argtypes = [C.POINTER(CertSpec), C.POINTER(Pair), C.c_int, C.c_int,
                                      C.c_int, C.c_int]
        L.mindist_calibrate.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_double),
                                        C.POINTER(C.c_double)]
        L.mindist_device.argtypes = [C.c_char_p, C.c_int, ip]
        L.mindist_peak_xorpop.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.mindist_walk_pair.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.POINTER(C.c_int32),
                                        u64p, C.POINTER(C.c_double)]
        if hasattr(L, "mindist_run_batch"):
            L.mindist_run_batch.argtypes = [C.POINTER(u64p), ip, ip, C.c_int,
                                            C.POINTER(Result), C.POINTER(BatchOpts)]
        if hasattr(L, "mindist_server_create"):
            L.mindist_server_create.argtypes = [C.POINTER(ServerOpts), C.POINTER(vp)]
            L.mindist_server_submit.argtypes = [vp, u64p, C.c_int, C.c_int, C.c_uint64]
            L.mindist_server_poll.argtypes = [vp, C.POINTER(ServerResult), C.c_int, ip]
            L.mindist_server_wait.argtypes = [vp, C.c_double]
            L.mindist_server_stats_get.argtypes = [vp, C.POINTER(ServerStats)]
            L.mindist_server_clock.argtypes = [vp]
            L.mindist_server_clock.restype = C.c_double
            L.mindist_server_destroy.argtypes = [vp]
            L.mindist_server_destroy.restype = None
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise MindistError(rc, lib().mindist_last_error().decode())
    return rc


def _mat(G, n, k):
    G = np.ascontiguousarray(G, dtype=np.uint64)
    if G.shape != (k, (n + 63) // 64):
        raise ValueError(f"G must have shape ({k}, {(n + 63) // 64}), got {G.shape}")
    return G


def _u64(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


def plan(G, n: int, k: int):
    """Host-only: (full sets, partial set, Gamma matrices) as the library builds them."""
    G = _mat(G, n, k)
    W = (n + 63) // 64
    sets = np.zeros(n, dtype=np.int32)
    mf, km = C.c_int(0), C.c_int(0)
    gam = np.zeros(((n // k) + 1) * k * W, dtype=np.uint64)
    _check(lib().mindist_plan(_u64(G), n, k, sets.ctypes.data_as(C.POINTER(C.c_int)),
                              C.byref(mf), C.byref(km), _u64(gam)))
    full = [sets[j * k:(j + 1) * k].tolist() for j in range(mf.value)]
    part = sets[mf.value * k: mf.value * k + km.value].tolist()
    ng = mf.value + (1 if km.value >= 1 else 0)
    return full, part, gam[:ng * k * W].reshape(ng, k, W).copy()


def calibrate(dwords: int = 3, blocks_per_cu: int = 4):
    """Measured ceiling of the enumeration's inner loop: (codewords/s, seconds)."""
    r, t = C.c_double(), C.c_double()
    _check(lib().mindist_calibrate(dwords, blocks_per_cu, C.byref(r), C.byref(t)))
    return r.value, t.value


PEAK_VARIANTS = 4


def peak_xorpop(variant: int = 1, blocks_per_cu: int = 8):
    """Measured register-only ceiling: (32-bit XOR+popcount ops/s, seconds)."""
    r, t = C.c_double(), C.c_double()
    _check(lib().mindist_peak_xorpop(variant, blocks_per_cu, C.byref(r), C.byref(t)))
    return r.value, t.value


def device() -> dict:
    """Architecture name and compute-unit count of the current GPU."""
    buf = C.create_string_buffer(64)
    cus = C.c_int(0)
    _check(lib().mindist_device(buf, 64, C.byref(cus)))
    return {"arch": buf.value.decode(), "compute_units": cus.value}


def colex_unrank(rank: int, r: int, hi: int) -> list:
    """Host-only: the r-subset of [0, hi) with colex rank `rank`, ascending."""
    out = (C.c_int * max(r, 1))()
    _check(lib().mindist_colex_unrank(rank, r, hi, out))
    return list(out[:r])


def bound_after(k, m_full, k_partial, include_partial, j, w) -> int:
    return _check(lib().mindist_bound_after(k, m_full, k_partial, int(include_partial), j, w))


def _policy(partial) -> int:
    return PARTIAL[partial] if isinstance(partial, str) else int(partial)


def schedule(k: int, m_full: int, k_partial: int, partial=0, per_level: bool = False) -> list:
    """Host-only: Algorithm 1's pairs up to level k as (j, w, g, L_after) tuples."""
    n = C.c_int(0)
    _check(lib().mindist_schedule(k, m_full, k_partial, _policy(partial), int(per_level), None, 0,
                                  C.byref(n)))
    out = (C.c_int32 * (4 * max(n.value, 1)))()
    _check(lib().mindist_schedule(k, m_full, k_partial, _policy(partial), int(per_level), out,
                                  n.value, C.byref(n)))
    return [tuple(out[4 * t:4 * t + 4]) for t in range(n.value)]


def certify(n: int, k: int, m_full: int, k_partial: int, pairs: list, d: int, L_final: int,
            exited_midpair: int = 0, partial=0, per_level: bool = False,
            midpair_exit: bool = True) -> int:
    """Host-only: run the library's certificate over a visited-pair trace
    (dicts with j, w, L_before, L_after, U_after, pair_min, count, executed).
    Returns 0; raises MindistError (E_CERT) when the trace fails it."""
    spec = CertSpec(n, k, m_full, k_partial, _policy(partial), int(per_level), int(midpair_exit))
    arr = (Pair * max(len(pairs), 1))()
    for t, p in enumerate(pairs):
        for f in ("j", "w", "L_before", "L_after", "U_after", "pair_min", "count", "executed"):
            setattr(arr[t], f, int(p[f]))
    return _check(lib().mindist_certify(C.byref(spec), arr, len(pairs), d, L_final, exited_midpair))


class MinDist:
    """One code: mindist_create / set_option / run / get_pairs / destroy."""

    def __init__(self, G, n: int, k: int, **options):
        self.n, self.k = n, k
        self._G = _mat(G, n, k)
        h = C.c_void_p()
        _check(lib().mindist_create(_u64(self._G), n, k, C.byref(h)))
        self._h = h
        for key, v in options.items():
            self.set_option(key, v)

    def set_option(self, key: str, value):
        if key == "partial":
            value = _policy(value)
        if key == "stream" and hasattr(value, "cuda_stream"):
            # a torch stream object
            if not _with_torch:
                raise MindistError(-1, "the library was loaded before torch: import torch "
                                       "first to share its HIP runtime and streams")
            value = value.cuda_stream
        _check(lib().mindist_set_option(self._h, OPT[key], int(value)))

    def info(self):
        mf, km, ng = C.c_int(), C.c_int(), C.c_int()
        _check(lib().mindist_info(self._h, C.byref(mf), C.byref(km), C.byref(ng)))
        return mf.value, km.value, ng.value

    def run(self) -> dict:
        r = Result()
        _check(lib().mindist_run(self._h, C.byref(r)))
        out = r.to_dict()
        out["pairs"] = self.pairs()
        return out

    def walk_pair(self, j: int, w: int, blocks_per_cu: int = 0) -> dict:
        """Pair (Gamma_j, w) by the lexicographic walk kernel (comparison only)."""
        pm, ex, sec = C.c_int32(), C.c_uint64(), C.c_double()
        _check(lib().mindist_walk_pair(self._h, j, w, blocks_per_cu, C.byref(pm), C.byref(ex),
                                       C.byref(sec)))
        return {"pair_min": pm.value, "executed": ex.value, "seconds": sec.value}

    def pairs(self):
        cnt = C.c_int()
        _check(lib().mindist_get_pairs(self._h, None, 0, C.byref(cnt)))
        arr = (Pair * max(cnt.value, 1))()
        _check(lib().mindist_get_pairs(self._h, arr, cnt.value, C.byref(cnt)))
        return _pair_dicts(arr, 0, cnt.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().mindist_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


BATCH_MAX_PAIRS = 256


def run_batch(codes, tile_min: int = 0, tile_max: int = 0, blocks_per_cu: int = 0,
              use_graph: int = 1, table_kib: int = 0, jobs_per_code: int = 0,
              pairs: bool = True, deadline_s: float = 60.0, chunks_per_visit: int = 0,
              direct_log2: int = 0):
    """Solve many codes in one call: short codes in one persistent launch,
    codes expected to enumerate at least 2^direct_log2 combinations (0 =
    2^30; -1 = none) through the single-code path on worker threads.

    codes: iterable of (n, k, G).  Returns (results, info): results[i] is the
    dict of mindist_run for code i (with "pairs" when requested) or
    {"error": code}; info holds the timings and the executed codeword count.
    """
    codes = list(codes)
    B = len(codes)
    mats = [_mat(G, n, k) for n, k, G in codes]
    ptrs = (C.POINTER(C.c_uint64) * B)(*[_u64(m) for m in mats])
    ns = (C.c_int * B)(*[n for n, _, _ in codes])
    ks = (C.c_int * B)(*[k for _, k, _ in codes])
    out = (Result * B)()
    o = BatchOpts()
    o.tile_min, o.tile_max, o.blocks_per_cu = tile_min, tile_max, blocks_per_cu
    o.use_graph, o.table_kib, o.jobs_per_code = use_graph, table_kib, jobs_per_code
    o.deadline_s = deadline_s
    o.chunks_per_visit = chunks_per_visit
    o.direct_log2 = direct_log2
    done = (C.c_double * B)()
    o.done_s = C.cast(done, C.c_void_p)
    if pairs:
        cap = B * BATCH_MAX_PAIRS
        # not zero-filled: the library writes every record the index names
        parr = (Pair * cap).from_buffer(np.empty(max(cap, 1) * C.sizeof(Pair), dtype=np.uint8))
        idx = (C.c_int64 * (B + 1))()
        o.pairs = C.cast(parr, C.c_void_p)
        o.pairs_cap = cap
        o.pairs_index = C.cast(idx, C.c_void_p)
    _check(lib().mindist_run_batch(ptrs, ns, ks, B, out, C.byref(o)))
    results = []
    for i in range(B):
        if out[i].d < 0:
            results.append({"error": out[i].d, "n": codes[i][0], "k": codes[i][1]})
            continue
        r = out[i].to_dict()
        if pairs:
            r["pairs"] = _pair_dicts(parr, idx[i], min(idx[i + 1], cap))
        results.append(r)
    info = {"seconds_kernel": o.seconds_kernel, "seconds_total": o.seconds_total,
            "seconds_prep": o.seconds_prep, "executed_total": o.executed_total,
            "wave_s_table": o.wave_s_table, "wave_s_pair": o.wave_s_pair,
            "wave_s_flush": o.wave_s_flush, "waves": o.waves,
            "chunks_table": o.chunks_table, "chunks_pair": o.chunks_pair,
            "done_s": list(done)}
    return results, info


class Server:
    """Continuous batching of arriving codes on the current GPU (the
    mindist_server_* entry points).  submit() returns at once; poll()
    returns finished results as dicts with the request's tag, its result,
    its visited pairs and t_submit / t_admit / t_done on the server clock.
    engine 0: worker threads running the single-code path side by side;
    engine 1: the persistent multi-code kernel, admitting codes while it
    runs, with codes above 2^route_log2 estimated combinations on
    single-path workers beside it."""

    def __init__(self, max_active: int = 0, blocks_per_cu: int = 0, device_bytes: int = 0,
                 epoch_min_ms: float = 0.0, table_kib: int = 0, jobs_per_code: int = 0,
                 chunks_per_visit: int = 0, engine: int = 0, linger_ms: float = 0.0,
                 route_log2: int = 0):
        o = ServerOpts(max_active, blocks_per_cu, device_bytes, epoch_min_ms, table_kib,
                       jobs_per_code, chunks_per_visit, engine, linger_ms, route_log2)
        h = C.c_void_p()
        _check(lib().mindist_server_create(C.byref(o), C.byref(h)))
        self._h = h
        self._buf = (ServerResult * 64)()

    def submit(self, G, n: int, k: int, tag: int):
        m = _mat(G, n, k)
        _check(lib().mindist_server_submit(self._h, _u64(m), n, k, tag))

    def poll(self) -> list:
        out = []
        while True:
            got = C.c_int(0)
            _check(lib().mindist_server_poll(self._h, self._buf, len(self._buf), C.byref(got)))
            for t in range(got.value):
                r = self._buf[t]
                d = {"tag": r.tag, "status": r.status, "t_submit": r.t_submit,
                     "t_admit": r.t_admit, "t_done": r.t_done}
                if r.status == 0:
                    d.update(r.result.to_dict())
                    d["pairs"] = _pair_dicts(r.pairs, 0, r.n_pairs)
                out.append(d)
            if got.value < len(self._buf):
                return out

    def wait(self, timeout_s: float = 60.0):
        _check(lib().mindist_server_wait(self._h, timeout_s))

    def clock(self) -> float:
        return lib().mindist_server_clock(self._h)

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().mindist_server_stats_get(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if self._h:
            lib().mindist_server_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_noalloc(G, n: int, k: int, stream: int = 0, pairs_cap: int = 4096) -> dict:
    """mindist_run_noalloc: one code through the single path with no device
    or pinned allocation (a fixed static device buffer per GPU)."""
    m = _mat(G, n, k)
    r = Result()
    arr = (Pair * pairs_cap)()
    cnt = C.c_int(0)
    _check(lib().mindist_run_noalloc(_u64(m), n, k, int(stream), C.byref(r), arr, pairs_cap,
                                     C.byref(cnt)))
    out = r.to_dict()
    out["pairs"] = _pair_dicts(arr, 0, min(cnt.value, pairs_cap))
    return out


def min_distance(G, n: int, k: int, **options) -> dict:
    with MinDist(G, n, k, **options) as m:
        return m.run()
