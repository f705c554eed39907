"""Benchmark: exact minimum distance of the seeded random [150,75] code on one GPU.

One step = the whole single-code path through the C ABI: mindist_create
(validate, pack, information sets, Gamma_j, device upload) + mindist_run
(Algorithm 1: every pair (Gamma_j, w) enumerated by the HIP kernel until
L >= U, witness rebuilt and checked) + mindist_destroy.  The input matrix
is generated before the timed region.

Prints one JSON line:
  value      codewords evaluated per second over the timed steps
  roofline   the enumeration kernel against the chip's 32-bit VALU peak:
             one codeword = D 32-bit XOR+popcount ops (D = words carried,
             3 for [150,75] with identity columns stripped), each op = 2 VALU
             lane instructions, peak = 256 CU x 64 lanes x 2.4 GHz / 2
  cpu_baseline  the CPU oracle (stack-based BZ enumeration, all threads it
             was given) on a bounded sample of the same pair
  batch      (if present) batched vs one-run-per-code codes/s
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_DWORD_OPS = 256 * 64 * 2.4e9 / 2      # 32-bit XOR+popcount per second
LANE_ITEMS = 4                              # left subsets per lane (library default)


def single_code_leg(steps: int, warmup: int):
    import paper_1603_06757_amd as md
    from paper_1603_06757_amd.gen import WORKLOADS

    w = WORKLOADS["rand150x75"]
    G = w.matrix()
    results = []

    def one():
        with md.MinDist(G, w.n, w.k, profile=1) as m:
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
    return w, results, t1 - t0


def roofline(results):
    # dominant kernel: the enumeration instance (dwords carried) with the most time
    per_d = {}
    for r in results:
        for p in r["pairs"]:
            t = per_d.setdefault(p["dwords"], [0.0, 0, 0])
            t[0] += p["ms"] * 1e-3
            t[1] += p["executed"]
            t[2] += 1
    D, (sec, cw, launches) = max(per_d.items(), key=lambda kv: kv[1][0])
    achieved = cw * D / sec
    return D, {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": PEAK_DWORD_OPS / 1e12,
        "unit": "T 32-bit xor+popcount/s",
        "frac": achieved / PEAK_DWORD_OPS,
        "traffic": None,
        "kernel": f"md::enum_pair_kernel<{D}, {LANE_ITEMS}, false>",
        "launches": launches,
        "avg_launch_us": sec / launches * 1e6,
        "ops_per_launch": cw * D / launches,
        "codewords_per_s_kernel": cw / sec,
    }


def cpu_baseline(w, seconds: float = 12.0):
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    G = w.matrix()
    full, _ = oracle.partition(G, w.n, w.k)
    Gam = oracle.gamma(G, w.n, w.k, full[0])
    end = oracle.binom(w.k, 8)
    lo, total, t_used = 0, 0, 0.0
    chunk = 1 << 25
    while t_used < seconds and lo < end:
        t = time.perf_counter()
        _, _, _, cnt, _ = oracle.pair(Gam, w.n, w.k, 8, lo, min(lo + chunk, end), threads)
        t_used += time.perf_counter() - t
        lo += chunk
        total += cnt
    return {"value": total / t_used, "unit": "codewords/s", "cores": threads, "kind": "oracle",
            "sample": f"pair (Gamma_1, w=8) of [{w.n},{w.k}], lexicographic ranks [0,{min(lo, end)}), "
                      f"{t_used:.1f}s, stack-based enumeration, full-width rows"}


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
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run plain device copies of this size (counter reference) and exit")
    a = ap.parse_args()
    if a.gpus != 1:
        print("this benchmark runs on one GPU only (single-GPU build); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    if a.copy_probe_mib:
        copy_probe(a.copy_probe_mib)
        return
    w, results, dt = single_code_leg(a.steps, a.warmup)
    ref = results[0]
    for r in results:
        assert r["d"] == ref["d"]
    executed = sum(r["executed_total"] for r in results)
    D, roof = roofline(results)
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
        "dtype": "u32",
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
    if not a.no_cpu:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
