"""The paper's CPU algorithm family (libmindist_cpu.so, Section 3) against
the oracle and the section's cost lemmas.

* Every algorithm returns the oracle's pair minimum and evaluates exactly
  C(k, w) combinations, on full and partial sets, w = 1 .. 7, several
  thread counts and saved levels s (so that 1, 2 and 3 chunks occur).
* Row additions follow the lemmas: basic C(k,w)(w-1); optimized
  C(k-1,w-1)(w-2) + C(k,w) (the count its proof derives; the printed
  statement's index shift gives smaller numbers, see the brute-force check
  below); stack C(k,w) + C(k-1,w-1) + ... + C(k-w+2,2); saved with s levels
  C(k,w) floor((w-1)/s) while w <= 2s (the prefix sums of longer splits are
  shared, so beyond 2s the count is at most that).  The closed forms are
  themselves checked against brute-force counting over all combinations.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1603_06757_amd import cpu
from paper_1603_06757_amd.gen import random_generator

ALGS = ["basic", "optimized", "stack", "saved", "saved_unroll2"]


def gammas(G, n, k):
    full, part = oracle.partition(G, n, k)
    return [oracle.gamma(G, n, k, s) for s in full + ([part] if part else [])]


@pytest.mark.parametrize("n,k,seed", [(40, 16, 1), (60, 20, 2), (70, 30, 3), (130, 24, 4)])
def test_family_matches_oracle(n, k, seed):
    G = random_generator(n, k, seed, 7)
    for g in gammas(G, n, k):
        for w in range(1, min(k, 7) + 1):
            ref = oracle.pair(g, n, k, w)[0]
            for alg in ALGS:
                for s in ((2, 3, 5) if alg.startswith("saved") else (5,)):
                    r = cpu.cpu_pair(g, k, w, alg, s=s, threads=3)
                    assert r["pair_min"] == ref, (n, k, w, alg, s)
                    assert r["combinations"] == math.comb(k, w), (n, k, w, alg, s)


def stack_lemma(k, w):
    return sum(math.comb(k - i, w - i) for i in range(0, w - 1)) if w >= 2 else 0


def optimized_count(k, w):
    return math.comb(k - 1, w - 1) * (w - 2) + math.comb(k, w) if w >= 2 else 0


def brute_counts(k, w):
    """Row additions by walking the combinations as each algorithm does."""
    basic = math.comb(k, w) * (w - 1)
    opt = stack = 0
    prev = None
    for pre in itertools.combinations(range(k - 1), w - 1):
        ext = k - 1 - pre[-1]              # last elements after the prefix
        opt += (w - 2) + ext
        if prev is None or prev[0] != pre[0]:
            changed = 1                    # a new first element: rebuild above it
        else:
            changed = next(i for i in range(w - 1) if pre[i] != prev[i])
        stack += (w - 1 - changed) + ext
        prev = pre
    return basic, opt, stack


@pytest.mark.parametrize("k,w", [(6, 3), (8, 4), (10, 5), (9, 2), (12, 6), (15, 4)])
def test_lemma_closed_forms_by_brute_force(k, w):
    basic, opt, stack = brute_counts(k, w)
    assert basic == math.comb(k, w) * (w - 1)
    assert opt == optimized_count(k, w)
    assert stack == stack_lemma(k, w)
    # four small cases counted by hand
    assert {(6, 3): 30, (8, 4): 140, (10, 5): 630, (9, 2): 36}.get((k, w), opt) == opt


@pytest.mark.parametrize("k,w,s", [(20, 2, 5), (20, 4, 5), (24, 6, 5), (24, 7, 3), (18, 5, 2),
                                   (30, 8, 4), (16, 9, 3)])
def test_family_addition_counts(k, w, s):
    rng = np.random.default_rng(k * 100 + w)
    rows = rng.integers(0, 2**63, size=(k, 2), dtype=np.uint64)
    C = math.comb(k, w)
    got = {a: cpu.cpu_pair(rows, k, w, a, s=s, threads=2) for a in ALGS}
    mins = {r["pair_min"] for r in got.values()}
    assert len(mins) == 1
    assert got["basic"]["additions"] == C * (w - 1)
    assert got["optimized"]["additions"] == optimized_count(k, w)
    assert got["stack"]["additions"] == stack_lemma(k, w)
    for a in ("saved", "saved_unroll2"):
        if w <= 2 * s:
            assert got[a]["additions"] == C * ((w - 1) // s), (a, k, w, s)
        else:
            assert got[a]["additions"] <= C * ((w - 1) // s), (a, k, w, s)
            assert got[a]["additions"] >= C, (a, k, w, s)


def test_family_brute_force_minimum():
    """Pair minima against a direct evaluation of every combination."""
    rng = np.random.default_rng(5)
    k = 14
    rows = rng.integers(0, 2**63, size=(k, 1), dtype=np.uint64)
    for w in range(1, 6):
        ref = min(bin(int(np.bitwise_xor.reduce(rows[list(c), 0]))).count("1")
                  for c in itertools.combinations(range(k), w))
        for a in ALGS:
            assert cpu.cpu_pair(rows, k, w, a, s=2, threads=1)["pair_min"] == ref, (w, a)
            assert cpu.cpu_pair(rows, k, w, a, s=2, offset=w)["pair_min"] == ref + w


def test_family_arguments():
    rows = np.zeros((4, 1), dtype=np.uint64)
    with pytest.raises(RuntimeError):
        cpu.cpu_pair(rows, 4, 5, "basic")
    with pytest.raises(RuntimeError):
        cpu.cpu_pair(rows, 4, 2, "saved", s=0)
    with pytest.raises(RuntimeError):
        cpu.cpu_pair(np.zeros((4, 9), dtype=np.uint64), 4, 2, "stack")
