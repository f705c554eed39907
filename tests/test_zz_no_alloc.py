"""mindist_run_noalloc (no device or pinned allocation: a fixed static
device buffer per GPU) against mindist_run, the entry point it is a variant
of, and against the oracle: two calls in a row, the second on a smaller
code, then more codes of other shapes, each compared exactly (d, the
visited pairs, bounds, minima, counts, executed combinations of completed
pairs) with a valid witness."""
import json
import os

import numpy as np
import pytest

import oracle
import paper_1603_06757_amd as md
from paper_1603_06757_amd.gen import WORKLOADS, random_generator
from tests import codes
from tests.test_gpu_parity import check_witness, compare_with_trace, oracle_tables

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print("[case]", *a, flush=True)


def same_run(a, b):
    assert a["d"] == b["d"]
    assert (a["m_full"], a["k_partial"], a["L_final"]) == (b["m_full"], b["k_partial"], b["L_final"])
    key = lambda p: (p["j"], p["w"], p["L_before"], p["L_after"], p["U_after"], p["pair_min"], p["count"])
    assert [key(p) for p in a["pairs"]] == [key(p) for p in b["pairs"]]
    for pa, pb in zip(a["pairs"][:-1], b["pairs"][:-1]):
        assert pa["executed"] == pb["executed"] == pa["count"]


def test_noalloc_equals_run_two_calls_second_smaller():
    big, small = WORKLOADS["rand150x75"], WORKLOADS["rand48x24"]
    for w in (big, small):
        G = w.matrix()
        say("noalloc", w.name, w.n, w.k)
        got = md.run_noalloc(G, w.n, w.k)
        ref = md.min_distance(G, w.n, w.k)
        same_run(got, ref)
        check_witness(G, w.n, w.k, got)
        gold = json.load(open(os.path.join(GOLDEN, f"{w.name}.json")))
        compare_with_trace(got, gold["trace"], gold["counts"], gold["pair_min"], None, w.k)


def test_noalloc_partial_sets_wide_rows_and_edges():
    w = WORKLOADS["rand255x40"]
    gold = json.load(open(os.path.join(GOLDEN, "rand255x40.json")))
    say("noalloc rand255x40")
    got = md.run_noalloc(w.matrix(), w.n, w.k)
    same_run(got, md.min_distance(w.matrix(), w.n, w.k))
    compare_with_trace(got, gold["trace"], gold["counts"], gold["pair_min"], None, w.k)
    check_witness(w.matrix(), w.n, w.k, got)
    cases = [codes.golay24(),
             codes.reed_muller(2, 8, True), codes.even_weight(64),
             (random_generator(512, 20, 512, 0), 512, 20), (random_generator(130, 1, 1, 130), 130, 1)]
    for G, n, k in cases:
        say("noalloc", n, k)
        got = md.run_noalloc(G, n, k)
        same_run(got, md.min_distance(G, n, k))
        check_witness(G, n, k, got)
        if k <= 24:
            r = oracle.bz(G, n, k, threads=4)
            counts, pmin, _ = oracle_tables(r)
            compare_with_trace(got, r["trace"].tolist(), counts, pmin, None, k)


def test_noalloc_pairs_cap_errors_and_reuse():
    w = WORKLOADS["rand48x24"]
    G = w.matrix()
    with md.MinDist(G, w.n, w.k) as m:
        ref = m.run()
    got = md.run_noalloc(G, w.n, w.k, pairs_cap=1)
    assert got["d"] == ref["d"] and len(got["pairs"]) == 1
    with pytest.raises(md.MindistError) as e:
        md.run_noalloc(np.zeros((3, 1), dtype=np.uint64), 3, 3)     # k = n
    assert e.value.code == -1
    R = np.array([[0b0011], [0b0110], [0b0101]], dtype=np.uint64)  # rank 2 < k = 3
    with pytest.raises(md.MindistError) as e:
        md.run_noalloc(R, 4, 3)
    assert e.value.code == -2
    # the buffer keeps the last call's contents; the next call is unaffected
    again = md.run_noalloc(G, w.n, w.k)
    assert again["d"] == ref["d"]
