"""GPU parity of the comparison kernel (mindist_walk_pair): the per-lane
lexicographic walk over one pair must give the CPU oracle's pair minimum and
evaluate exactly C(k, w) combinations, for full (identity-stripped) and
partial sets, every w up to its limit, ragged lane ranges and several launch
shapes; out-of-range requests are refused with MINDIST_E_LIMIT / E_ARG."""
import math
import sys

import pytest

import oracle
import paper_1603_06757_amd as md
from paper_1603_06757_amd.gen import WORKLOADS, random_generator
from tests import codes

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def gammas(G, n, k):
    full, part = oracle.partition(G, n, k)
    return [oracle.gamma(G, n, k, s) for s in full + ([part] if part else [])]


def check_code(G, n, k, ws, bpc=0):
    gam = gammas(G, n, k)
    with md.MinDist(G, n, k) as m:
        for j, g in enumerate(gam):
            for w in ws:
                if w > k:
                    continue
                r = m.walk_pair(j, w, bpc)
                ref = oracle.pair(g, n, k, w, threads=8)[0]
                assert r["pair_min"] == ref, (n, k, j, w, r, ref)
                assert r["executed"] == math.comb(k, w), (n, k, j, w, r)


def test_walk_48x24_every_w():
    w = WORKLOADS["rand48x24"]
    say("walk rand48x24 w 1..12")
    check_code(w.matrix(), w.n, w.k, range(1, 13))


def test_walk_150x75_low_w():
    w = WORKLOADS["rand150x75"]
    say("walk rand150x75 w 1..5")
    check_code(w.matrix(), w.n, w.k, range(1, 6))


@pytest.mark.parametrize("bpc", [1, 8])
def test_walk_partial_set_and_shapes(bpc):
    G = random_generator(100, 40, 11, 0)
    full, part = oracle.partition(G, 100, 40)
    assert len(full) == 2 and len(part) > 0
    say("walk [100,40] with a partial set, blocks per CU", bpc)
    check_code(G, 100, 40, range(1, 6), bpc)


def test_walk_single_combination_and_textbook():
    G, n, k = codes.golay24()
    say("walk golay24, w = k = 12")
    check_code(G, n, k, [1, 2, 11, 12])
    G, n, k = codes.hamming7()
    check_code(G, n, k, range(1, 5))


def test_walk_matches_main_path_pair_minima():
    w = WORKLOADS["rand150x75"]
    say("walk vs mindist_run pair minima on rand150x75, w <= 6")
    with md.MinDist(w.matrix(), w.n, w.k) as m:
        res = m.run()
        for p in res["pairs"]:
            if p["w"] <= 6 and p["executed"] == p["count"]:
                r = m.walk_pair(p["j"], p["w"])
                assert r["pair_min"] == p["pair_min"], (p, r)


def test_walk_limits():
    w = WORKLOADS["rand255x40"]                  # 7 carried words per row
    say("walk limits")
    with md.MinDist(w.matrix(), w.n, w.k) as m:
        with pytest.raises(md.MindistError) as e:
            m.walk_pair(0, 3)
        assert e.value.code == -5
    w = WORKLOADS["rand48x24"]
    with md.MinDist(w.matrix(), w.n, w.k) as m:
        for j, ww, code in ((0, 13, -5), (0, 0, -1), (0, 25, -1), (5, 2, -1)):
            with pytest.raises(md.MindistError) as e:
                m.walk_pair(j, ww)
            assert e.value.code == code, (j, ww)
