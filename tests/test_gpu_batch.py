"""GPU parity of the multi-code path: the persistent launch, and the single
path for the long codes a batch routes there.

Every code of a batch must give exactly what the single-code path gives with
default options (d, the visited pairs, every pair minimum, the counts C(k,w),
the bounds before and after each pair), and on small codes what the CPU
oracle gives; witnesses may differ but must be valid.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
import paper_1603_06757_amd as md
from paper_1603_06757_amd.gen import WORKLOADS, batch_code, random_generator, PCG32, draw_matrix
from tests import codes
from tests.test_gpu_parity import check_witness, compare_with_trace, oracle_tables, estimated_work

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print("[case]", *a, flush=True)


def same_as_single(r, s):
    assert r["d"] == s["d"]
    key = lambda p: (p["j"], p["w"], p["L_before"], p["U_after"], p["pair_min"], p["count"])
    assert [key(p) for p in r["pairs"]] == [key(p) for p in s["pairs"]]
    for pr, ps in zip(r["pairs"], s["pairs"]):
        if pr["executed"] == pr["count"] and ps["executed"] == ps["count"]:
            assert pr["L_after"] == ps["L_after"]


def light_codes(count, seed=77):
    """Seeded random codes the oracle solves quickly, within the batch limits
    (n <= 256, at most 32 information sets)."""
    rng = PCG32(seed, 11)
    out = []
    while len(out) < count:
        n = rng.uniform_int(10, 200)
        k = rng.uniform_int(1, min(n - 1, 64))
        if estimated_work(n, k) > 3e7:
            continue
        G = draw_matrix(rng, n, k)
        try:
            full, part = oracle.partition(G, n, k)
        except oracle.OracleError:
            continue
        if len(full) + (1 if part else 0) > 32:
            continue
        out.append((n, k, G))
    return out


def test_batch_matches_oracle_small_codes():
    cs = light_codes(160)
    say("batch of", len(cs), "light random codes")
    res, info = md.run_batch(cs)
    errs = [(n, k, r.get("error")) for (n, k, G), r in zip(cs, res) if "error" in r]
    assert not errs, errs
    for (n, k, G), r in zip(cs, res):
        ref = oracle.bz(G, n, k, threads=4)
        assert r["d"] == ref["d"], (n, k)
        counts, pmin, ws = oracle_tables(ref)
        compare_with_trace(r, ref["trace"].tolist(), counts, pmin, None, k)
        check_witness(G, n, k, r)


@pytest.mark.parametrize("direct_log2", [0, -1])
def test_batch_workloads_and_textbook_golden(direct_log2):
    """The long codes go through the single path by default (direct_log2 = 0)
    and through the persistent launch with -1; both match the goldens."""
    names = ["rand48x24", "rand150x75", "rand255x40", "golay24", "rm_2_7", "rm_3_7",
             "rm_2_8", "rm_2_8_punct"]
    ctors = {"golay24": codes.golay24, "rm_2_7": lambda: codes.reed_muller(2, 7),
             "rm_3_7": lambda: codes.reed_muller(3, 7), "rm_2_8": lambda: codes.reed_muller(2, 8),
             "rm_2_8_punct": lambda: codes.reed_muller(2, 8, True)}
    cs = []
    for nm in names:
        if nm in WORKLOADS:
            w = WORKLOADS[nm]
            cs.append((w.n, w.k, w.matrix()))
        else:
            G, n, k = ctors[nm]()
            cs.append((n, k, G))
    say("batch of workloads + textbook codes, direct_log2", direct_log2)
    res, info = md.run_batch(cs, direct_log2=direct_log2)
    for nm, (n, k, G), r in zip(names, cs, res):
        gold = json.load(open(os.path.join(GOLDEN, f"{nm}.json")))
        assert r["d"] == gold["d"], nm
        compare_with_trace(r, gold["trace"], gold["counts"], gold["pair_min"], None, k)
        check_witness(G, n, k, r)


def test_batch_equals_single_on_batch_stream():
    """The first 256 codes of the 4096-code batch stream whose work is light."""
    cs = []
    i = 0
    while len(cs) < 200:
        n, k, G = batch_code(i)
        i += 1
        if estimated_work(n, k) <= 5e9:
            cs.append((n, k, G))
    say("batch stream subset", len(cs))
    res, info = md.run_batch(cs)
    for (n, k, G), r in zip(cs, res):
        s = md.min_distance(G, n, k)
        same_as_single(r, s)
        check_witness(G, n, k, r)


@pytest.mark.parametrize("graph,tmin,tmax,bpc", [(0, 256, 2048, 4), (1, 64, 256, 2), (1, 1024, 1024, 5)])
def test_batch_launch_shapes(graph, tmin, tmax, bpc):
    cs = light_codes(48, seed=5)
    say("launch shape", graph, tmin, tmax, bpc)
    res, info = md.run_batch(cs, use_graph=graph, tile_min=tmin, tile_max=tmax, blocks_per_cu=bpc,
                             direct_log2=-1)
    for (n, k, G), r in zip(cs, res):
        ref = oracle.bz(G, n, k, threads=4)
        assert r["d"] == ref["d"]
        counts, pmin, ws = oracle_tables(ref)
        compare_with_trace(r, ref["trace"].tolist(), counts, pmin, None, k)


def test_batch_errors_reported_per_code():
    good = light_codes(3, seed=9)
    dep = codes.pack(np.array([[1, 0, 1, 1], [1, 0, 1, 1]], dtype=np.uint8))
    cs = good[:1] + [(4, 2, dep)] + good[1:]
    say("batch with a rank-deficient code")
    res, info = md.run_batch(cs)
    assert res[1]["error"] == -2
    for (n, k, G), r in zip([cs[0], cs[2], cs[3]], [res[0], res[2], res[3]]):
        assert r["d"] == oracle.bz(G, n, k)["d"]


def test_batch_limits_reported():
    """More than 32 information sets is beyond the persistent launch's
    layout: E_LIMIT for that code when every code must run there, the
    single path's answer when routing is on; the others unaffected."""
    G = random_generator(200, 3, 1, 2)
    good = light_codes(2, seed=13)
    res, info = md.run_batch([(200, 3, G)] + good, direct_log2=-1)
    assert res[0]["error"] == -5
    for (n, k, G2), r in zip(good, res[1:]):
        assert r["d"] == oracle.bz(G2, n, k)["d"]
    res, info = md.run_batch([(200, 3, G)] + good)
    assert res[0]["d"] == oracle.bz(G, 200, 3)["d"]
    same_as_single(res[0], md.min_distance(G, 200, 3))


@pytest.mark.parametrize("direct_log2", [0, -1])
def test_batch_single_code_and_repeat(direct_log2):
    w = WORKLOADS["rand150x75"]
    gold = json.load(open(os.path.join(GOLDEN, "rand150x75.json")))
    for _ in range(3):
        res, info = md.run_batch([(w.n, w.k, w.matrix())], direct_log2=direct_log2)
        assert res[0]["d"] == gold["d"]
        compare_with_trace(res[0], gold["trace"], gold["counts"], gold["pair_min"], None, w.k)


def test_batch_kernel_keeps_two_blocks_per_cu():
    """The persistent kernel must fit 2 blocks of 256 threads per CU (at
    most 256 VGPRs, the matrix-core inner loop's budget): a larger register
    budget silently halves the resident waves."""
    cs = light_codes(4, seed=95)
    res, info = md.run_batch(cs, direct_log2=-1)
    say("waves", info["waves"])
    assert info["waves"] == 256 * 2 * 4      # MI355X: 256 CUs, 2 blocks of 4 waves


def test_batch_routes_long_codes_to_the_single_path():
    """A mixed batch: short codes share the persistent launch, long ones (and
    one beyond the launch's limits) run through the single path on worker
    threads; every result equals the code's single run, in input order."""
    light = light_codes(40, seed=96)
    w150, w255 = WORKLOADS["rand150x75"], WORKLOADS["rand255x40"]
    wide = random_generator(200, 3, 1, 2)
    cs = light[:20] + [(w150.n, w150.k, w150.matrix())] + light[20:] + \
        [(w255.n, w255.k, w255.matrix()), (200, 3, wide)]
    say("mixed batch", len(cs))
    res, info = md.run_batch(cs)
    assert info["waves"] > 0                 # the persistent launch ran
    for (n, k, G), r in zip(cs, res):
        same_as_single(r, md.min_distance(G, n, k))
        check_witness(G, n, k, r)
    assert all(x >= 0 for x in info["done_s"])
