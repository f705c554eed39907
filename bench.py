"""Benchmark: exact minimum distance of the seeded random [150,75] code on one GPU.

One step = the whole single-code path through the C ABI: mindist_create
(validate, pack, information sets, Gamma_j, device upload) + mindist_run
(Algorithm 1: every pair (Gamma_j, w) enumerated by the HIP kernel until
L >= U, witness rebuilt and certified) + mindist_destroy.  The input matrix
is generated before the timed region.

Prints one JSON line:
  value      codewords evaluated per second over the timed steps
  roofline   the dominant enumeration kernel against the VALU ceiling: one
             codeword = D 32-bit XOR+popcount ops (D = words carried, 3 for
             [150,75] with identity columns stripped); peak = the larger of
             the rated-clock figure (256 CU x 64 lanes x 2.4 GHz / 2) and
             the measured register-only ceiling (mindist_peak_xorpop)
  time_to_d  the whole path on [48,24], [255,40] (median of repeats) and
             [150,75] (the timed steps), with the share of the VALU peak
  section6   the smallest Section 6 code, [232,51], certified (d = 61 claimed)
  serving    open-loop Poisson arrivals of the serving stream at 10, 30, 100,
             300 and 1000 per second under both engines: p50/p99 latency
             (all and by work), codes/s, offered load, requests left out by
             the work cap
  cpu_baseline  the CPU oracle (stack-based BZ enumeration) on the host's
             threads (at most 16) and on one thread, median of 3 windows;
             brute force and the oracle's BZ on [48,24]
  batch      all 4096 codes of the batch stream: one mindist_run per code,
             one mindist_run_batch call (long codes routed to the single
             path) and one persistent launch for every code, results
             compared in full; per-stratum speed-ups
--new-codes certifies the codes of Section 6 instead (one line per code);
--compare-walk measures the saved-sums kernel against the direct walk;
--cpu-family times the paper's CPU algorithms on the host (Table 1's code size);
--peak runs the register-only ceiling kernel alone.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_DWORD_OPS = 256 * 64 * 2.4e9 / 2      # derived: 32-bit XOR+popcount per second at the rated clock
LANE_ITEMS = 4                              # left subsets per lane (library default)
MFMA_MAX_WORDS = 4                          # widest codeword the matrix-core inner loop takes


def single_code_leg(steps: int, warmup: int):
    import paper_1603_06757_amd as md
    from paper_1603_06757_amd.gen import WORKLOADS

    w = WORKLOADS["rand150x75"]
    G = w.matrix()
    results = []

    def one(profile=0):
        with md.MinDist(G, w.n, w.k, profile=profile) as m:
            r = m.run()
        return r

    for i in range(warmup):
        one()
        print(f"[bench] warmup {i + 1}/{warmup} done", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for i in range(steps):
        results.append(one())
    t1 = time.perf_counter()
    print(f"[bench] timed {steps} steps in {t1 - t0:.3f}s", file=sys.stderr, flush=True)
    # untimed: the same runs with HIP events around every enumeration launch
    # (each event adds a few microseconds between kernels, so they stay out
    # of the timed steps); their kernel times cross-check the device clock
    events = [one(profile=1) for _ in range(2)]
    return w, results, t1 - t0, events


KERNEL_SOURCES = ["paper_1603_06757_amd/csrc/mindist_kernels.hip",
                  "paper_1603_06757_amd/csrc/mindist_device.h",
                  "paper_1603_06757_amd/csrc/mindist_internal.h"]
COUNTERS = os.path.join(ROOT, "profiles", "enum_pair_kernel_rand150x75_counters.txt")


def measured_traffic():
    """HBM bytes per launch of the enumeration kernel from the committed
    counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's
    reading), or None once the kernel sources differ from the ones the
    counters were taken with."""
    import hashlib
    try:
        text = open(COUNTERS).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    vals = dict(line.split(":", 1) for line in text.splitlines()
                if line.startswith(("traffic_bytes_per_launch:", "kernel_sources_sha256_16:")))
    if vals.get("kernel_sources_sha256_16", "").split()[:1] != [h.hexdigest()[:16]]:
        return None
    return float(vals["traffic_bytes_per_launch"])


PEAK_INT8_OPS = 5.0e15                      # MI355X dense int8 matrix-core peak, ops/s


def roofline(results, events, peak, mfma=True):
    """peak: the larger of the derived figure and the measured register-only
    ceiling, in 32-bit XOR+popcount ops/s.  mfma: the library's default
    inner loop for codewords of at most 4 words, a 32 x 32 x 32 int8 product
    per word (64 D ops per codeword) priced against the int8 matrix-core
    peak; the vector-ALU figures stay beside it."""
    # dominant kernel: the enumeration instance (dwords carried) with the most
    # time.  Launch times of the timed steps come from the device clock (the
    # kernel's first wave start to its last wave end, published with each
    # pair); HIP events on the kernel's stream in untimed runs cross-check them.
    def per_dwords(runs, field):
        # per launch (short consecutive pairs share one): its pairs start
        # together, so its time is the longest of theirs; codewords add up
        per_d = {}
        for r in runs:
            launches = {}
            for p in r["pairs"]:
                t = launches.setdefault(p["launch"], [p["dwords"], 0.0, 0])
                t[1] = max(t[1], p[field] * 1e-3)
                t[2] += p["executed"]
            for D, sec, cw in launches.values():
                t = per_d.setdefault(D, [0.0, 0, 0])
                t[0] += sec
                t[1] += cw
                t[2] += 1
        return per_d
    per_d = per_dwords(results, "dev_ms")
    D, (sec, cw, launches) = max(per_d.items(), key=lambda kv: kv[1][0])
    ev_sec, ev_cw, ev_launches = per_dwords(events, "ms").get(D, (0.0, 0, 0))
    achieved = cw * D / sec
    on_mfma = mfma and D <= MFMA_MAX_WORDS
    roof = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": peak / 1e12,
        "unit": "T 32-bit xor+popcount/s",
        "frac": achieved / peak,
        "peak_nominal": PEAK_DWORD_OPS / 1e12,
        "frac_nominal": achieved / PEAK_DWORD_OPS,
        "peak_source": "measured register-only ceiling (mindist_peak_xorpop, best shape and occupancy)"
                       if peak > PEAK_DWORD_OPS else "derived: 256 CU x 64 lanes x 2.4 GHz / 2",
    }
    if on_mfma:
        ops = cw * 64 * D / sec
        roof = {
            "bound": "mfma",
            "achieved": ops / 1e12,
            "peak": PEAK_INT8_OPS / 1e12,
            "unit": "TOP/s (int8)",
            "frac": ops / PEAK_INT8_OPS,
            "ops_per_codeword": 64 * D,
            "peak_source": "MI355X dense int8 matrix-core peak",
            # the same launches as XOR+popcount work, against the vector-ALU ceiling
            "xorpop_equiv": achieved / 1e12,
            "xorpop_equiv_unit": "T 32-bit xor+popcount/s",
            "xorpop_equiv_over_valu_peak": achieved / peak,
            "valu_peak": peak / 1e12,
            "valu_peak_nominal": PEAK_DWORD_OPS / 1e12,
        }
    roof.update({
        "traffic": measured_traffic(),
        "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
        "kernel": f"md::enum_pair_kernel<{D}, {LANE_ITEMS}, false, {'true' if on_mfma else 'false'}>",
        "launches": launches,
        "avg_launch_us": sec / launches * 1e6,
        "timing": "device clock per launch in the timed steps; HIP events in 2 untimed runs",
        "avg_launch_us_events": ev_sec / ev_launches * 1e6 if ev_launches else None,
        "codewords_per_s_kernel_events": ev_cw / ev_sec if ev_sec else None,
        "ops_per_launch": cw * (64 * D if on_mfma else D) / launches,
        "codewords_per_s_kernel": cw / sec,
    })
    return D, roof


def cpu_baseline(w, seconds: float = 4.0, repeats: int = 3):
    """The CPU oracle on the host: its stack-based enumeration of pair
    (Gamma_1, w=8) of [150,75] over windows of consecutive lexicographic
    ranks, on every host thread this process may use (at most 16, the GPU
    box's share) and on one thread, median of `repeats` windows of about
    `seconds` each; plus brute force over all 2^24 messages of [48,24] and
    the oracle's whole BZ run on it, one thread."""
    import statistics
    import oracle
    from paper_1603_06757_amd.gen import WORKLOADS
    nproc = os.cpu_count() or 1
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = nproc
    threads = max(1, min(usable, 16))
    G = w.matrix()
    full, _ = oracle.partition(G, w.n, w.k)
    Gam = oracle.gamma(G, w.n, w.k, full[0])
    end = oracle.binom(w.k, 8)

    def window(th, r):
        # window r starts at rank r * end / repeats and runs about `seconds`
        lo, hi = r * end // repeats, (r + 1) * end // repeats
        total, t_used = 0, 0.0
        chunk = 1 << (25 if th > 1 else 22)
        while t_used < seconds and lo < hi:
            t = time.perf_counter()
            _, _, _, cnt, _ = oracle.pair(Gam, w.n, w.k, 8, lo, min(lo + chunk, hi), th)
            t_used += time.perf_counter() - t
            lo += chunk
            total += cnt
        return total / t_used, total, t_used

    runs = {}
    for th in (threads, 1):
        rs = [window(th, r) for r in range(repeats)]
        runs[th] = rs
        print(f"[bench] cpu oracle, {th} threads: {statistics.median(r[0] for r in rs):.3e} codewords/s",
              file=sys.stderr, flush=True)
    med = lambda th: statistics.median(r[0] for r in runs[th])
    c1 = WORKLOADS["rand48x24"]
    G1 = c1.matrix()
    t = time.perf_counter()
    d_brute, _, _ = oracle.brute(G1, c1.n, c1.k)
    t_brute = time.perf_counter() - t
    t = time.perf_counter()
    r1 = oracle.bz(G1, c1.n, c1.k, threads=1)
    t_bz1 = time.perf_counter() - t
    assert r1["d"] == d_brute
    return {"value": med(threads), "unit": "codewords/s", "cores": threads, "kind": "oracle",
            "sample": f"pair (Gamma_1, w=8) of [{w.n},{w.k}]: {repeats} windows of consecutive "
                      f"lexicographic ranks, ~{seconds:.0f} s each, median; stack-based enumeration, "
                      f"full-width rows",
            "nproc": nproc, "usable_cpus": usable,
            "single_thread": {"value": med(1), "unit": "codewords/s", "cores": 1},
            "windows": {str(th): [{"codewords": c, "seconds": s_} for _, c, s_ in rs]
                        for th, rs in runs.items()},
            "config1_brute_force": {"code": "[48,24]", "d": d_brute, "messages": 2 ** c1.k,
                                    "seconds": t_brute, "threads": 1,
                                    "codewords_per_s": (2 ** c1.k) / t_brute},
            "config1_oracle_bz": {"code": "[48,24]", "d": r1["d"], "seconds": t_bz1, "threads": 1}}


def time_to_d_leg(peak: float, repeats=(("rand48x24", 30), ("rand255x40", 10))):
    """Time to d of the small and the low-rate single codes: the whole path
    (mindist_create + mindist_run + mindist_destroy) per run, median of the
    repeats, and the share of the VALU peak over that whole time (each
    pair's evaluated codewords times its 32-bit words)."""
    import statistics
    import paper_1603_06757_amd as md
    from paper_1603_06757_amd.gen import WORKLOADS
    out = {}
    for name, reps in repeats:
        w = WORKLOADS[name]
        G = w.matrix()
        md.min_distance(G, w.n, w.k)             # warm: shapes, pools
        times, r = [], None
        for _ in range(reps):
            t0 = time.perf_counter()
            r = md.min_distance(G, w.n, w.k)
            times.append(time.perf_counter() - t0)
        t = statistics.median(times)
        ops = sum(p["executed"] * p["dwords"] for p in r["pairs"])
        out[name] = {"n": w.n, "k": w.k, "d": r["d"], "pairs": r["pairs_visited"],
                     "codewords": r["executed_total"], "time_to_d_ms": t * 1e3,
                     "time_to_d_ms_min": min(times) * 1e3, "runs": reps,
                     "codewords_per_s": r["executed_total"] / t, "valu_frac": ops / t / peak}
        print(f"[bench] time to d {name}: {t * 1e3:.3f} ms", file=sys.stderr, flush=True)
    return out


def estimated_work(md, G, n: int, k: int) -> float:
    """Codewords Algorithm 1 is expected to evaluate on a random [n,k] code:
    the pair sequence's bound against the Gilbert-Varshamov distance (the
    smallest d with sum_{i<=d} C(n,i) >= 2^(n-k)), summing C(k,w) per pair.
    Used only to stratify and cap synthetic workloads."""
    import math
    full, part, _ = md.plan(G, n, k)
    mf, km = len(full), len(part)
    ng = mf + (1 if km >= 1 else 0)
    acc, d = 0, n - k + 1
    for i in range(n + 1):
        acc += math.comb(n, i)
        if acc >= 2 ** (n - k):
            d = i
            break
    f = lambda i, h: h + 1 if i < mf else max(0, h + 1 - (k - km))
    L, work = 1, 0.0
    for w in range(1, k + 1):
        for j in range(ng):
            if L >= d:
                return work
            work += math.comb(k, w)
            L = sum(f(i, w if i <= j else w - 1) for i in range(ng))
    return work


# work strata of the batch stream, by the codewords a code's run evaluates
STRATA = (("light", 0.0, 1e9), ("medium", 1e9, 2e10), ("heavy", 2e10, 1e12),
          ("very_heavy", 1e12, float("inf")))


def _pair_key(p):
    return (p["j"], p["w"], p["L_before"], p["U_after"], p["pair_min"], p["count"])


def _same_runs(a, b) -> bool:
    """d, the whole visited-pair sequence (set, level, bound before, U after,
    pair minimum, C(k,w)), and L after and executed for every completed pair."""
    if a.get("d") != b.get("d") or len(a["pairs"]) != len(b["pairs"]):
        return False
    for pa, pb in zip(a["pairs"], b["pairs"]):
        if _pair_key(pa) != _pair_key(pb):
            return False
        if pa["executed"] == pa["count"] and pb["executed"] == pb["count"] and pa["L_after"] != pb["L_after"]:
            return False
    return all(pa["executed"] == pb["executed"] for pa, pb in zip(a["pairs"][:-1], b["pairs"][:-1]))


def batch_leg(codes_total: int, stride: int, strata_calls=("light", "medium", "heavy")):
    """The batch stream (every `stride`-th code; 1 = all): one mindist_run
    per code (each timed), the whole stream in one mindist_run_batch call
    with long codes routed to the single path, and in one persistent launch
    for every code; every code's result compared in full.  Strata by the
    codewords each code evaluates; the strata in `strata_calls` are also run
    as batches of their own, for per-stratum speed-ups."""
    import paper_1603_06757_amd as md
    from paper_1603_06757_amd.gen import batch_code
    from paper_1603_06757_amd.autotune import tuned_options
    idx = list(range(0, codes_total, stride))
    codes = [batch_code(i) for i in idx]
    say = lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True)

    def tuning_sample():
        # other codes of the same stream, without the heaviest (tuning in seconds)
        out = []
        for i in range(4, codes_total, 32):
            n, k, G = batch_code(i)
            if estimated_work(md, G, n, k) <= 2e11:
                out.append((n, k, G))
        return out

    t0 = time.perf_counter()
    opts = tuned_options(f"batch stream of {codes_total} codes", tuning_sample, log=say)
    t_tune = time.perf_counter() - t0
    md.run_batch(codes[:4], pairs=False, **opts)
    # one run per code, each timed
    plain, t_plain = [], []
    t0 = t_say = time.perf_counter()
    for i, (n, k, G) in enumerate(codes):
        t = time.perf_counter()
        plain.append(md.min_distance(G, n, k))
        t_plain.append(time.perf_counter() - t)
        if time.perf_counter() - t_say > 15:
            say(f"one run per code: {i + 1}/{len(codes)}")
            t_say = time.perf_counter()
    tp = time.perf_counter() - t0
    say(f"one run per code: {tp:.2f}s")
    stratum = []
    for r in plain:
        for name, lo, hi in STRATA:
            if lo <= r["executed_total"] < hi:
                stratum.append(name)
                break
    # the whole stream, routed and persistent-only
    t0 = time.perf_counter()
    res, info = md.run_batch(codes, pairs=True, deadline_s=400, **opts)
    tb = time.perf_counter() - t0
    say(f"batch of {len(codes)} codes, long codes routed: {tb:.2f}s")
    t0 = time.perf_counter()
    res_p, info_p = md.run_batch(codes, pairs=True, deadline_s=400, direct_log2=-1, **opts)
    tpers = time.perf_counter() - t0
    say(f"batch of {len(codes)} codes, one persistent launch: {tpers:.2f}s")
    same = [_same_runs(r, p) for r, p in zip(res, plain)]
    same_p = [_same_runs(q, p) for q, p in zip(res_p, plain)]
    strata = {}
    for name, lo, hi in STRATA:
        members = [i for i, s_ in enumerate(stratum) if s_ == name]
        if not members:
            continue
        rec = {"codewords_range": [lo, hi if hi != float("inf") else None], "codes": len(members),
               "codewords": sum(plain[i]["executed_total"] for i in members),
               "plain_s": sum(t_plain[i] for i in members)}
        rec["codes_per_s_plain"] = len(members) / rec["plain_s"]
        if name in strata_calls:
            sub = [codes[i] for i in members]
            for mode, kw in (("routed", {}), ("persistent_only", {"direct_log2": -1})):
                t0 = time.perf_counter()
                sr, _ = md.run_batch(sub, pairs=True, deadline_s=400, **kw, **opts)
                dt = time.perf_counter() - t0
                rec[f"{mode}_s"] = dt
                rec[f"codes_per_s_{mode}"] = len(sub) / dt
                rec[f"speedup_{mode}"] = rec["plain_s"] / dt
                rec[f"identical_{mode}"] = all(_same_runs(a, plain[i]) for a, i in zip(sr, members))
            say(f"stratum {name}: {len(members)} codes, plain {rec['plain_s']:.2f}s, "
                f"routed {rec['routed_s']:.2f}s, persistent {rec['persistent_only_s']:.2f}s")
        else:
            rec["note"] = "not run as a batch of its own: its codes dominate the whole-stream calls"
        strata[name] = rec
    return {"codes": len(codes), "sample": f"codes 0,{stride},...,{codes_total - stride} of the "
                                            f"{codes_total}-code stream" if stride > 1 else
                                            f"all {codes_total} codes",
            "plain_s": tp, "codes_per_s_plain": len(codes) / tp,
            "batched_s": tb, "codes_per_s_batched": len(codes) / tb, "speedup": tp / tb,
            "persistent_only_s": tpers, "codes_per_s_persistent_only": len(codes) / tpers,
            "speedup_persistent_only": tp / tpers,
            "identical": all(same), "identical_codes": sum(same),
            "identical_persistent_only": all(same_p), "identical_codes_persistent_only": sum(same_p),
            "identity": "d and the whole visited-pair sequence (set, level, L before, U after, pair "
                        "minimum, C(k,w); L after and executed of completed pairs) against one "
                        "mindist_run per code",
            "routing": "codes estimated at >= 2^30 combinations through the single path "
                       "on 8 worker threads, the rest in one persistent launch",
            "strata": strata,
            "kernel_s": info["seconds_kernel"], "kernel_s_persistent_only": info_p["seconds_kernel"],
            "autotuned": opts, "autotune_s": t_tune,
            "codewords": sum(r["executed_total"] for r in plain),
            "codewords_per_s_plain": sum(r["executed_total"] for r in plain) / tp}


SERVING_STRATA = (("under_1e7", 0.0, 1e7), ("1e7_to_1e9", 1e7, 1e9), ("1e9_to_cap", 1e9, float("inf")))


def serving_leg(rate: float, seconds: float, cap: float, max_requests: int = 4000, engine: int = 0,
                rate_codewords: float = 0.0):
    """Open-loop Poisson arrivals of the serving stream at `rate` per second
    for about `seconds`; requests whose estimated work exceeds `cap`
    codewords are left out of the stream (counted in the report).  engine 0:
    worker threads running the single-code path side by side; engine 1: the
    persistent multi-code kernel.  Latency = completion - submission;
    offered load = rate x the mean evaluated codewords per request /
    rate_codewords (the single path's codewords/s)."""
    import numpy as np
    import paper_1603_06757_amd as md
    from paper_1603_06757_amd.gen import serving_request, poisson_arrivals
    want = min(max_requests, max(8, int(rate * seconds)))
    kept, skipped, i = [], 0, 0
    while len(kept) < want:
        n, k, G = serving_request(i)
        i += 1
        if estimated_work(md, G, n, k) > cap:
            skipped += 1
            continue
        kept.append((n, k, G))
    arr = poisson_arrivals(len(kept), rate)
    with md.Server(engine=engine) as srv:
        t_start = time.perf_counter()
        for tag, (t, (n, k, G)) in enumerate(zip(arr, kept)):
            dt = t - (time.perf_counter() - t_start)
            if dt > 0:
                time.sleep(dt)
            srv.submit(G, n, k, tag=tag)
        got, t_say = [], time.perf_counter()
        while len(got) < len(kept) and time.perf_counter() - t_start < 300:
            got += srv.poll()
            if time.perf_counter() - t_say > 5.0:
                print(f"[bench] serving {rate}/s engine {engine}: {len(got)}/{len(kept)} done",
                      file=sys.stderr, flush=True)
                t_say = time.perf_counter()
            time.sleep(0.002)
        t_end = max(r["t_done"] for r in got) - min(r["t_submit"] for r in got) if got else 0.0
        st = srv.stats()
    lat = np.array([r["t_done"] - r["t_submit"] for r in got]) if got else np.zeros(1)
    ok = [r for r in got if r["status"] == 0]
    work = [r["executed_total"] for r in ok]
    mean_work = float(np.mean(work)) if work else 0.0
    per = {}
    for name, lo, hi in SERVING_STRATA:
        ls = [r["t_done"] - r["t_submit"] for r in ok if lo <= r["executed_total"] < hi]
        if ls:
            per[name] = {"requests": len(ls), "p50_ms": float(np.percentile(ls, 50) * 1e3),
                         "p99_ms": float(np.percentile(ls, 99) * 1e3)}
    return {"engine": engine, "rate_per_s": rate, "requests": len(kept), "completed_ok": len(ok),
            "skipped_over_cap": skipped, "work_cap_codewords": cap,
            "offered_s": float(arr[-1]), "wall_s": t_end,
            "codes_per_s": len(got) / t_end if t_end else 0.0,
            "mean_codewords": mean_work,
            "offered_load": rate * mean_work / rate_codewords if rate_codewords else None,
            "latency_p50_ms": float(np.percentile(lat, 50) * 1e3),
            "latency_p99_ms": float(np.percentile(lat, 99) * 1e3),
            "by_work": per, "epochs": st["epochs"], "admitted_live": st["admitted_live"],
            "routed": st["routed"],
            "kernel_s": st["seconds_kernel"]}


SERVING_RATES = ((10, 8.0), (30, 4.0), (100, 2.5), (300, 1.5), (1000, 1.0))


def serving_sweep(cap: float, rate_codewords: float, engines=(0, 1), rates=SERVING_RATES):
    out = {}
    for engine in engines:
        out[f"engine{engine}"] = [serving_leg(r, sec, cap, engine=engine, rate_codewords=rate_codewords)
                                  for r, sec in rates]
    return out


# Section 6's timings of its best CPU implementation (vectorised saved
# additions) on its own machine, seconds on 1 core and on 6 cores: context
# for the GPU times, not a target measured here.
PAPER_CPU_S = {
    "mp235x51": (234890.8, 38428.5),
    "mp236x51": (231345.5, 38497.1),
    "mp233x51": (159470.8, 26725.6),
    "mp233x52": (225141.2, 37660.1),
    "mp232x51": (125695.6, 20691.6),
}


def new_codes_leg(names, quiet: bool = False, peak: float = 0.0):
    """Section 6's codes through the single-code path, one fresh context
    each: d against the claimed distance, time, codewords and the share of
    the VALU peak (every pair's codewords times its 32-bit words)."""
    import paper_1603_06757_amd as md
    from paper_1603_06757_amd.newcodes import NEW_CODES
    out = []
    for name in names or list(NEW_CODES):
        c = NEW_CODES[name]
        G = c.matrix()
        print(f"[bench] section 6 code {name} [{c.n},{c.k}]", file=sys.stderr, flush=True)
        t0 = time.perf_counter()
        r = md.min_distance(G, c.n, c.k)
        dt = time.perf_counter() - t0
        ops = sum(p["executed"] * p["dwords"] for p in r["pairs"])
        rec = {"new_code": name, "n": c.n, "k": c.k, "d": r["d"], "d_claimed": c.d,
               "d_previously_known": c.d_before, "certified": r["d"] == c.d,
               "seconds": dt, "pairs": r["pairs_visited"], "codewords": r["executed_total"],
               "codewords_per_s": r["executed_total"] / dt,
               "valu_frac": ops / dt / max(peak, PEAK_DWORD_OPS),
               "ops_per_s": ops / dt}
        if name in PAPER_CPU_S:
            one, six = PAPER_CPU_S[name]
            rec["paper_cpu_s"] = {"1_core": one, "6_cores": six}
        out.append(rec)
        if not quiet:
            print(json.dumps(rec), flush=True)
    return out


def walk_compare_leg(repeats: int = 3):
    """The saved-sums kernel against the per-lane lexicographic walk
    (mindist_walk_pair) on the same pairs of [150,75]: codewords/s of each,
    the walk's best of `repeats` launches, the saved-sums kernel's pair time
    from the device clock in a full run."""
    import paper_1603_06757_amd as md
    from paper_1603_06757_amd.gen import WORKLOADS
    w = WORKLOADS["rand150x75"]
    out = []
    with md.MinDist(w.matrix(), w.n, w.k) as m:
        m.run()                                   # tables and shapes built
        res = m.run()
        for p in res["pairs"]:
            if p["w"] < 6 or p["executed"] != p["count"]:
                continue
            best = None
            for _ in range(repeats):
                r = m.walk_pair(p["j"], p["w"])
                assert r["pair_min"] == p["pair_min"] and r["executed"] == p["count"]
                best = r["seconds"] if best is None else min(best, r["seconds"])
            saved = p["count"] / (p["dev_ms"] * 1e-3)
            walk = p["count"] / best
            rec = {"walk_compare": f"[{w.n},{w.k}] pair (j={p['j']}, w={p['w']})",
                   "combinations": p["count"], "dwords": p["dwords"],
                   "saved_sums_codewords_per_s": saved, "walk_codewords_per_s": walk,
                   "saved_over_walk": saved / walk,
                   "walk_frac_of_peak": walk * p["dwords"] / PEAK_DWORD_OPS}
            out.append(rec)
            print(json.dumps(rec), flush=True)
    return out


# Table 1: the whole run on the paper's random [150,50,28], one core, seconds
PAPER_TABLE1_S = {
    "basic": (511.5, 273.1), "optimized": (191.0, 105.3), "stack": (144.5, 84.6),
    "saved": (89.8, 44.7), "saved_unroll2": (74.0, 44.6),
}


def cpu_family_leg(threads: int = 0):
    """The paper's CPU algorithms (libmindist_cpu.so) over the pairs that
    Algorithm 1 visits on the seeded [150,50] stand-in with d = 28 (the GPU
    run gives the pair list and the minima they must reproduce), on the
    host's cores, next to Table 1's one-core times."""
    import paper_1603_06757_amd as md
    from paper_1603_06757_amd import cpu
    from paper_1603_06757_amd.gen import paper_random_code
    n, k, attempt = 150, 50, 4
    G = paper_random_code(n, k, attempt)
    md.min_distance(G, n, k)
    t0 = time.perf_counter()
    r = md.min_distance(G, n, k)
    t_gpu = time.perf_counter() - t0
    full, part, gam = md.plan(G, n, k)
    threads = threads or min(16, os.cpu_count() or 1)
    out, t_basic = [], None
    for alg in cpu.ALGORITHMS:
        t0 = time.perf_counter()
        tables = adds = combos = 0
        for p in r["pairs"]:
            c = cpu.cpu_pair(gam[p["j"]], k, p["w"], alg, s=5, threads=threads)
            if p["executed"] == p["count"]:
                assert c["pair_min"] == p["pair_min"], (alg, p)
            assert c["pair_min"] >= r["d"]
            tables += c["table_seconds"]
            adds += c["additions"]
            combos += c["combinations"]
        dt = time.perf_counter() - t0
        t_basic = t_basic or dt
        rec = {"cpu_family": alg, "code": f"[{n},{k}] d={r['d']} (seed 6, stream {1000 * n + k}, attempt {attempt})",
               "pairs": len(r["pairs"]), "threads": threads, "seconds": dt,
               "table_seconds": tables, "combinations": combos, "additions": adds,
               "codewords_per_s": combos / dt, "speedup_vs_basic": t_basic / dt,
               "paper_table1_1_core_s": {"cplex_opteron_6128": PAPER_TABLE1_S[alg][0],
                                         "marbore_xeon_e5_2695v3": PAPER_TABLE1_S[alg][1]},
               "paper_speedup_vs_basic_cplex": PAPER_TABLE1_S["basic"][0] / PAPER_TABLE1_S[alg][0],
               "gpu_seconds_same_code": t_gpu}
        out.append(rec)
        print(json.dumps(rec), flush=True)
    return out


def peak_leg(blocks_per_cu=(4, 8, 16)):
    """The measured register-only XOR+popcount ceiling (mindist_peak_xorpop):
    every loop shape at several occupancies; the best is the roofline's
    measured peak."""
    import paper_1603_06757_amd as md
    out = []
    for v in range(md.PEAK_VARIANTS):
        for b in blocks_per_cu:
            ops, sec = md.peak_xorpop(v, b)
            out.append({"variant": v, "blocks_per_cu": b, "ops_per_s": ops, "seconds": sec,
                        "over_derived": ops / PEAK_DWORD_OPS})
            print(f"[bench] peak kernel variant {v}, {b} blocks/CU: {ops / 1e12:.2f} T ops/s",
                  file=sys.stderr, flush=True)
    best = max(out, key=lambda r: r["ops_per_s"])
    return {"ops_per_s": best["ops_per_s"], "variant": best["variant"],
            "blocks_per_cu": best["blocks_per_cu"], "runs": out}


def batch_stratum_leg(name: str, codes_total: int = 4096):
    """One work stratum of the batch stream (by estimated codewords: light
    < 1e9, medium < 2e10, heavy < 1e12) in one persistent launch, once (a
    profiling target)."""
    import paper_1603_06757_amd as md
    from paper_1603_06757_amd.gen import batch_code
    lo, hi = {"light": (0, 1e9), "medium": (1e9, 2e10), "heavy": (2e10, 1e12)}[name]
    codes = [c for c in (batch_code(i) for i in range(codes_total)) if lo <= estimated_work(md, c[2], c[0], c[1]) < hi]
    t0 = time.perf_counter()
    res, info = md.run_batch(codes, pairs=True, direct_log2=-1, deadline_s=300)
    dt = time.perf_counter() - t0
    # 32-bit XOR + popcount operations: every pair's codewords times the
    # words its set carries
    ops = sum(p["executed"] * p["dwords"] for r in res if "error" not in r for p in r["pairs"])
    print(json.dumps({"batch_stratum": name, "codes": len(codes), "seconds": dt,
                      "kernel_s": info["seconds_kernel"], "codewords": info["executed_total"],
                      "dword_ops": ops, "dword_ops_per_s_kernel": ops / info["seconds_kernel"],
                      "errors": sum(1 for r in res if "error" in r)}), flush=True)


def copy_probe(mib: int):
    """Plain device-to-device copies of a known size: the reference reading
    for the FETCH_SIZE / WRITE_SIZE counters (each copy reads and writes
    mib MiB)."""
    import torch
    n = mib << 20
    x = torch.randint(0, 255, (n,), dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    print(json.dumps({"copy_probe_mib": mib, "copies": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--batch-stratum", choices=["light", "medium", "heavy"], default=None,
                    help="only run one work stratum of the batch stream in one persistent launch and exit")
    ap.add_argument("--peak", action="store_true",
                    help="only run the register-only XOR+popcount ceiling kernel and exit")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run plain device copies of this size (counter reference) and exit")
    ap.add_argument("--batch-codes", type=int, default=4096, help="size of the batch stream")
    ap.add_argument("--batch-stride", type=int, default=1,
                    help="batch leg: every stride-th code of the stream (1 = all, the default)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batch leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-section6", action="store_true",
                    help="skip certifying the smallest Section 6 code ([232,51,61], ~4 s)")
    ap.add_argument("--serving-sweep", action="store_true",
                    help="only run the serving sweep (one JSON line per arrival rate) and exit")
    ap.add_argument("--serving-cap", type=float, default=2e10,
                    help="serving: leave out requests above this many estimated codewords")
    ap.add_argument("--cpu-family", action="store_true",
                    help="only time the paper's CPU algorithms (libmindist_cpu.so) on the "
                         "seeded [150,50,28] code's pairs, next to Table 1, and exit")
    ap.add_argument("--compare-walk", action="store_true",
                    help="only compare the saved-sums kernel with the lexicographic walk "
                         "kernel on the pairs of [150,75] with w >= 6, and exit")
    ap.add_argument("--new-codes", nargs="*", default=None,
                    help="only certify Section 6's codes (all, or the names given; "
                         "one JSON line per code) and exit")
    a = ap.parse_args()
    if a.gpus != 1:
        print("this benchmark runs on one GPU only (single-GPU build); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if a.batch_stratum:
        batch_stratum_leg(a.batch_stratum)
        return
    if a.peak:
        print(json.dumps({"peak_xorpop": peak_leg()}), flush=True)
        return
    if a.copy_probe_mib:
        copy_probe(a.copy_probe_mib)
        return
    if a.cpu_family:
        cpu_family_leg()
        return
    if a.compare_walk:
        walk_compare_leg()
        return
    if a.new_codes is not None:
        new_codes_leg(a.new_codes)
        return
    if a.serving_sweep:
        for engine in (0, 1):
            for rate in (10, 30, 100, 300, 1000, 3000):
                if engine == 1 and rate > 1000:
                    continue           # already saturated at 1000/s
                print(json.dumps({"serving": serving_leg(rate, 4.0 if rate >= 100 else 10.0,
                                                         a.serving_cap, engine=engine,
                                                         rate_codewords=5.5e12)}), flush=True)
        return
    w, results, dt, events = single_code_leg(a.steps, a.warmup)
    ref = results[0]
    for r in results:
        assert r["d"] == ref["d"]
    executed = sum(r["executed_total"] for r in results)
    print("[bench] measured peak", file=sys.stderr, flush=True)
    peak = peak_leg()
    D, roof = roofline(results, events, max(PEAK_DWORD_OPS, peak["ops_per_s"]))
    roof["peak_measured"] = peak["ops_per_s"] / 1e12
    roof["peak_measured_shape"] = {"variant": peak["variant"], "blocks_per_cu": peak["blocks_per_cu"]}
    line = {
        "metric": "codewords/s (XOR+popcount) & time-to-d, [150,75]; batched vs plain codes/s",
        "value": executed / dt,
        "unit": "codewords/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": dt / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8" if roof["bound"] == "mfma" else "u32",
        "data": "synthetic",
        "config": {"workload": f"random [{w.n},{w.k}] binary code, PCG32 seed {w.seed} "
                               f"attempt {w.attempt}, Bernoulli(1/2), 2 information sets",
                   "d": ref["d"], "pairs": ref["pairs_visited"],
                   "codewords_per_step": ref["executed_total"],
                   "canonical_codewords": ref["canonical_total"],
                   "dwords_per_codeword": D,
                   "parallelism": "single GPU"},
        "time_to_d_ms": dt / a.steps * 1e3,
        "roofline": roof,
    }
    print("[bench] time to d, configs [48,24] and [255,40]", file=sys.stderr, flush=True)
    line["time_to_d"] = time_to_d_leg(max(PEAK_DWORD_OPS, peak["ops_per_s"]))
    line["time_to_d"]["rand150x75"] = {"time_to_d_ms": dt / a.steps * 1e3, "d": ref["d"],
                                       "valu_frac": sum(p["executed"] * p["dwords"] for r in results
                                                        for p in r["pairs"]) / dt
                                       / max(PEAK_DWORD_OPS, peak["ops_per_s"])}
    if not a.no_section6:
        print("[bench] section 6 code", file=sys.stderr, flush=True)
        line["section6"] = new_codes_leg(["mp232x51"], quiet=True, peak=peak["ops_per_s"])[0]
    if not a.no_serving:
        print("[bench] serving sweep", file=sys.stderr, flush=True)
        line["serving"] = serving_sweep(a.serving_cap, executed / dt)
    if not a.no_cpu:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w)
    if not a.no_batch:
        print("[bench] batch leg", file=sys.stderr, flush=True)
        line["batch"] = batch_leg(a.batch_codes, max(1, a.batch_stride))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
