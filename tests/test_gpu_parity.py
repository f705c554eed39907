"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Exact integer work, so the bar is bit-exactness: d, the visited pairs and
their order, every pair minimum, the canonical counts C(k,w), the bounds
before and after each pair, and (verify mode) every pair's weight sum.  A
witness is valid if it has weight d, is the XOR of the rows it names, and
lies in the row space of G.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

import oracle
import paper_1603_06757_amd as md
from paper_1603_06757_amd.gen import WORKLOADS, random_generator, PCG32, draw_matrix, batch_code
from tests import codes

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def rank_bits(bits):
    M = bits.copy() % 2
    r = 0
    for c in range(M.shape[1]):
        piv = np.nonzero(M[r:, c])[0]
        if len(piv) == 0:
            continue
        p = r + piv[0]
        M[[r, p]] = M[[p, r]]
        rows = np.nonzero(M[:, c])[0]
        for i in rows:
            if i != r:
                M[i] ^= M[r]
        r += 1
        if r == M.shape[0]:
            break
    return r


def check_witness(G, n, k, res):
    W = (n + 63) // 64
    bits = codes.unpack(res["witness"].reshape(1, W), n)[0]
    assert int(bits.sum()) == res["d"], "witness weight differs from d"
    Gb = codes.unpack(G, n)
    assert rank_bits(np.vstack([Gb, bits])) == k, "witness outside the row space"
    full, part, gam = md.plan(G, n, k)
    j, w = res["witness_pair"]
    assert len(res["witness_rows"]) == w
    acc = np.zeros(W, dtype=np.uint64)
    for r in res["witness_rows"]:
        acc ^= gam[j][r]
    assert (acc == res["witness"]).all()


def compare_with_trace(res, trace, counts, pair_min, wsum=None, k=None):
    """res: GPU result dict; trace rows (j, g, L_before, L_after, U_after, pair_min)."""
    gp = res["pairs"]
    assert len(gp) == len(trace), f"visited {len(gp)} pairs, oracle {len(trace)}"
    for p, t in zip(gp, trace):
        j, g, Lb, La, U, pm = t
        key = f"{j},{g}"
        assert (p["j"], p["w"]) == (j, g)
        assert p["L_before"] == Lb, (key, p["L_before"], Lb)
        assert p["pair_min"] == pm, (key, p["pair_min"], pm)
        assert p["U_after"] == U, (key, p["U_after"], U)
        assert p["count"] == counts[key] == math.comb(k, g)
        if p["executed"] == p["count"]:
            assert p["L_after"] == La, (key, p["L_after"], La)
        if wsum is not None and p["executed"] == p["count"]:
            assert p["wsum"] == wsum[key], (key, p["wsum"], wsum[key])


def oracle_tables(r):
    counts = {f"{j},{g}": int(r["counts"][j, g]) for j, g in r["trace"][:, :2].tolist()}
    pmin = {f"{j},{g}": int(r["pair_min"][j, g]) for j, g in r["trace"][:, :2].tolist()}
    ws = {f"{j},{g}": int(r["wsum"][j, g]) for j, g in r["trace"][:, :2].tolist()}
    return counts, pmin, ws


POLICY_NAMES = {0: "always", 1: "never", 2: "when_useful"}


def run_and_compare(G, n, k, verify=True, **opts):
    partial = opts.get("partial", 0)
    pname = partial if isinstance(partial, str) else POLICY_NAMES[int(partial)]
    r = oracle.bz(G, n, k, threads=4, per_level=bool(opts.get("term", 0)), partial=pname)
    res = md.min_distance(G, n, k, verify=int(verify), **opts)
    assert res["d"] == r["d"]
    assert res["m_full"] == r["m_full"] and res["k_partial"] == r["k_m"]
    counts, pmin, ws = oracle_tables(r)
    compare_with_trace(res, r["trace"].tolist(), counts, pmin, ws if verify else None, k)
    check_witness(G, n, k, res)
    return res, r


# ---------------------------------------------------------------- textbook
@pytest.mark.parametrize("name,ctor,d", [
    ("hamming7", codes.hamming7, 3),
    ("golay24", codes.golay24, 8),
    ("rm_1_5", lambda: codes.reed_muller(1, 5), 16),
    ("rm_2_6", lambda: codes.reed_muller(2, 6), 16),
    ("rm_1_6_punct", lambda: codes.reed_muller(1, 6, True), 31),
    ("repetition9", lambda: codes.repetition(9), 9),
    ("even_weight12", lambda: codes.even_weight(12), 2),
])
def test_textbook_small(name, ctor, d):
    G, n, k = ctor()
    say(name, n, k)
    res, r = run_and_compare(G, n, k)
    assert res["d"] == d


@pytest.mark.parametrize("name,d", [("golay24", 8), ("rm_2_7", 32), ("rm_3_7", 16),
                                    ("rm_2_8", 64), ("rm_2_8_punct", 63)])
def test_textbook_golden(name, d):
    gold = json.load(open(os.path.join(GOLDEN, f"{name}.json")))
    ctor = {"golay24": codes.golay24, "rm_2_7": lambda: codes.reed_muller(2, 7),
            "rm_3_7": lambda: codes.reed_muller(3, 7), "rm_2_8": lambda: codes.reed_muller(2, 8),
            "rm_2_8_punct": lambda: codes.reed_muller(2, 8, True)}[name]
    G, n, k = ctor()
    say(name, n, k)
    res = md.min_distance(G, n, k, verify=1)
    assert res["d"] == gold["d"] == d
    compare_with_trace(res, gold["trace"], gold["counts"], gold["pair_min"], gold["wsum"], k)
    check_witness(G, n, k, res)


# ---------------------------------------------------------------- workloads
@pytest.mark.parametrize("name", ["rand48x24", "rand150x75", "rand255x40"])
@pytest.mark.parametrize("verify", [0, 1])
def test_workload_golden(name, verify):
    gold = json.load(open(os.path.join(GOLDEN, f"{name}.json")))
    w = WORKLOADS[name]
    G = w.matrix()
    say(name, "verify", verify)
    res = md.min_distance(G, w.n, w.k, verify=verify)
    assert res["d"] == gold["d"]
    assert (res["m_full"], res["k_partial"]) == (gold["m_full"], gold["k_m"])
    compare_with_trace(res, gold["trace"], gold["counts"], gold["pair_min"],
                       gold["wsum"] if verify else None, w.k)
    assert res["canonical_total"] == gold["codewords"]
    check_witness(G, w.n, w.k, res)


def test_workload_48x24_brute():
    w = WORKLOADS["rand48x24"]
    G = w.matrix()
    d_b, _, _ = oracle.brute(G, w.n, w.k)
    say("rand48x24 brute")
    assert md.min_distance(G, w.n, w.k)["d"] == d_b


def test_midpair_exit_changes_only_executed():
    w = WORKLOADS["rand150x75"]
    G = w.matrix()
    say("rand150x75 midpair on/off")
    on = md.min_distance(G, w.n, w.k, midpair_exit=1)
    off = md.min_distance(G, w.n, w.k, midpair_exit=0)
    assert on["d"] == off["d"]
    assert [(p["j"], p["w"], p["pair_min"], p["count"]) for p in on["pairs"]] == \
           [(p["j"], p["w"], p["pair_min"], p["count"]) for p in off["pairs"]]
    assert all(p["executed"] == p["count"] for p in off["pairs"])
    assert all(p["executed"] == p["count"] for p in on["pairs"][:-1])
    assert on["pairs"][-1]["executed"] <= on["pairs"][-1]["count"]


def test_determinism_repeated_runs():
    w = WORKLOADS["rand255x40"]
    G = w.matrix()
    say("rand255x40 x5")
    with md.MinDist(G, w.n, w.k, midpair_exit=0) as m:
        ref = m.run()
        for _ in range(4):
            r = m.run()
            assert r["d"] == ref["d"]
            assert [(p["pair_min"], p["executed"]) for p in r["pairs"]] == \
                   [(p["pair_min"], p["executed"]) for p in ref["pairs"]]
            check_witness(G, w.n, w.k, r)


def test_launch_ahead_off_and_on_match_the_oracle():
    """Pairs launched ahead of their results (several while the queued work
    is short) change nothing a run reports: the same visited pairs, bounds,
    minima and counts as with no pair launched ahead, and as the oracle."""
    for i in range(12):
        n = 40 + 8 * (i % 5)
        k = n // 2 - (i % 3)
        G = random_generator(n, k, 700 + i)
        say("launch ahead", i, n, k)
        off, _ = run_and_compare(G, n, k, verify=False, speculate=0)
        on, _ = run_and_compare(G, n, k, verify=False)
        key = lambda r: [(p["j"], p["w"], p["pair_min"], p["L_before"]) for p in r["pairs"]]
        assert key(off) == key(on)
        # executed differs only where mid-pair exit cut the last pair
        assert [p["executed"] for p in off["pairs"][:-1]] == [p["executed"] for p in on["pairs"][:-1]]


def test_short_pairs_share_launches():
    """Short consecutive pairs run in one launch: each record names the
    first pair of its launch, launches hold consecutive pairs, at least one
    holds several on [150,75]; with nothing launched ahead every pair has
    its own launch.  The visited pairs are the same either way."""
    w = WORKLOADS["rand150x75"]
    G = w.matrix()
    say("rand150x75 launches")
    r = md.min_distance(G, w.n, w.k)
    launch = [p["launch"] for p in r["pairs"]]
    assert launch[0] == 0
    for i, l in enumerate(launch):
        assert l <= i and (i == 0 or l in (launch[i - 1], i))
    assert len(set(launch)) < len(launch)
    off = md.min_distance(G, w.n, w.k, speculate=0)
    assert [p["launch"] for p in off["pairs"]] == list(range(len(off["pairs"])))
    key = lambda x: [(p["j"], p["w"], p["pair_min"], p["L_before"], p["L_after"]) for p in x["pairs"]]
    assert key(r) == key(off) and r["d"] == off["d"]


def test_device_clock_pair_times_agree_with_events():
    """Every pair reports its kernel's span on the device clock (first wave
    start to last wave end); it is positive and no longer than the HIP-event
    time around the same launch, which adds only the dispatch."""
    w = WORKLOADS["rand150x75"]
    G = w.matrix()
    say("rand150x75 device clock vs events")
    with md.MinDist(G, w.n, w.k, profile=1) as m:
        m.run()
        r = m.run()
    big = 0
    for p in r["pairs"]:
        assert p["dev_ms"] > 0, p
        assert p["dev_ms"] <= p["ms"] + 0.005, p
        if p["ms"] > 1.0:
            big += 1
            assert p["dev_ms"] >= 0.95 * p["ms"], p
    assert big >= 1


# ---------------------------------------------------------------- random sweep
def estimated_work(n, k):
    """Rough oracle work of a random [n,k] code: d from the expected weight
    distribution C(n,w)/2^(n-k), level from the bound with floor(n/k) sets."""
    acc, d = 0, n
    for w in range(1, n + 1):
        acc += math.comb(n, w)
        if acc >= 2 ** (n - k):
            d = w + 2
            break
    m = max(1, n // k)
    g = 1
    while m * (g + 1) < d and g < k:
        g += 1
    return (m + 1) * sum(math.comb(k, t) for t in range(1, g + 1))


def test_random_codes_vs_oracle():
    """240 seeded codes, W = 1..4 words, k up to 64, both termination rules."""
    rng = PCG32(2024, 3)
    done = 0
    i = 0
    while done < 240:
        i += 1
        n = rng.uniform_int(10, 250)
        k = rng.uniform_int(1, min(n - 1, 64))
        if estimated_work(n, k) > 3e7:
            continue
        G = draw_matrix(rng, n, k)
        try:
            oracle.partition(G, n, k)
        except oracle.OracleError:
            continue
        say("random", i, n, k)
        run_and_compare(G, n, k, verify=(i % 3 == 0), term=i % 2,
                        midpair_exit=(i % 4 != 1), partial={4: 1, 2: 2}.get(i % 5, 0))
        done += 1


@pytest.mark.parametrize("tile_t,bpc", [(1, 1), (7, 2), (64, 8), (333, 3), (4096, 4)])
def test_tile_shapes(tile_t, bpc):
    for name in ["rand48x24", "rand150x75"]:
        gold = json.load(open(os.path.join(GOLDEN, f"{name}.json")))
        w = WORKLOADS[name]
        if name == "rand150x75" and tile_t < 64:
            continue
        say(name, "tile", tile_t, bpc)
        res = md.min_distance(w.matrix(), w.n, w.k, tile_t=tile_t, blocks_per_cu=bpc, verify=1)
        compare_with_trace(res, gold["trace"], gold["counts"], gold["pair_min"], gold["wsum"], w.k)


@pytest.mark.parametrize("order,counters,items,left", [(0, 1, 4, 1), (0, 8, 2, 0), (1, 8, 4, 1),
                                                       (1, 1, 2, 1), (1, 1, 4, 0)])
def test_chunk_orders_and_dispensers(order, counters, items, left):
    for name in ["rand48x24", "rand150x75", "rand255x40"]:
        gold = json.load(open(os.path.join(GOLDEN, f"{name}.json")))
        w = WORKLOADS[name]
        say(name, "order", order, "counters", counters, "items", items, "left tables", left)
        res = md.min_distance(w.matrix(), w.n, w.k, chunk_order=order, counters=counters,
                              lane_items=items, left_tables=left, verify=1)
        compare_with_trace(res, gold["trace"], gold["counts"], gold["pair_min"], gold["wsum"], w.k)


@pytest.mark.parametrize("mfma,items,order,tile_t", [(1, 4, 0, 0), (1, 2, 1, 0), (1, 4, 0, 33),
                                                    (1, 2, 0, 1024), (1, 4, 1, 100), (0, 4, 0, 0)])
def test_matrix_core_and_vector_inner_loops(mfma, items, order, tile_t):
    """Two-level pairs of 1 to 4 words per codeword with the inner loop on the
    int8 matrix cores (whole 32-entry blocks of the range every lane subset
    covers; the rest on the vector ALUs) or on the vector ALUs alone: d, every
    pair minimum, bound and count equal the oracle's.  Tile lengths of 33 and
    100 leave a ragged block in every chunk; 5 or more words always take the
    vector ALUs."""
    for name in ["rand48x24", "rand150x75", "rand255x40"]:
        gold = json.load(open(os.path.join(GOLDEN, f"{name}.json")))
        w = WORKLOADS[name]
        say(name, "mfma", mfma, "items", items, "order", order, "tile", tile_t)
        res = md.min_distance(w.matrix(), w.n, w.k, verify=0, mfma=mfma, lane_items=items,
                              chunk_order=order, tile_t=tile_t)
        compare_with_trace(res, gold["trace"], gold["counts"], gold["pair_min"], None, w.k)
        check_witness(w.matrix(), w.n, w.k, res)
    rng = PCG32(1603, 19 + mfma)
    for words in (1, 2, 3, 4):
        done = 0
        while done < 4:
            k = rng.uniform_int(6, 40)
            n = k + rng.uniform_int(32 * (words - 1) + 1, 32 * words)
            if estimated_work(n, k) > 3e7:
                continue
            G = draw_matrix(rng, n, k)
            try:
                oracle.partition(G, n, k)
            except oracle.OracleError:
                continue
            say("random", words, "words", n, k, "mfma", mfma)
            run_and_compare(G, n, k, verify=False, mfma=mfma, lane_items=items, chunk_order=order,
                            tile_t=tile_t)
            done += 1


@pytest.mark.parametrize("table_mib", [1, 2])
def test_three_level_split_small_tables(table_mib):
    """Small saved tables force the three-level split (lane subset, outer
    table, inner table) on the larger levels of [255,40], whose two-level
    right runs become short; results must not change."""
    for name in ["rand48x24", "rand150x75", "rand255x40"]:
        gold = json.load(open(os.path.join(GOLDEN, f"{name}.json")))
        w = WORKLOADS[name]
        say(name, "table_mib", table_mib)
        res = md.min_distance(w.matrix(), w.n, w.k, table_mib=table_mib, verify=1)
        assert any(p["split_b2"] > 0 for p in res["pairs"]) or name != "rand255x40"
        compare_with_trace(res, gold["trace"], gold["counts"], gold["pair_min"], gold["wsum"], w.k)
        check_witness(w.matrix(), w.n, w.k, res)
    rng = PCG32(31337, 5)
    done = 0
    while done < 40:
        n = rng.uniform_int(40, 200)
        k = rng.uniform_int(10, min(n - 1, 60))
        if estimated_work(n, k) > 3e7:
            continue
        G = draw_matrix(rng, n, k)
        try:
            oracle.partition(G, n, k)
        except oracle.OracleError:
            continue
        say("random small tables", n, k)
        run_and_compare(G, n, k, verify=True, table_mib=table_mib)
        done += 1


def test_max_width_code():
    """n = 512 (8 words, 16 dwords per row), many information sets."""
    G = random_generator(512, 20, 512, 0)
    say("random 512x20")
    run_and_compare(G, 512, 20)


def test_k1_and_small_edges():
    for n in (2, 3, 64, 65, 130, 512):
        G = random_generator(n, 1, 1, n)
        if not G.any():
            continue
        say("k=1 n", n)
        run_and_compare(G, n, 1)
    G, n, k = codes.even_weight(64)   # k = n-1: one full set and a rank-1 partial set
    say("even weight 64")
    run_and_compare(G, n, k)


def test_zero_and_repeated_columns():
    G, n, k = codes.golay24()
    b = codes.with_extra_columns(codes.unpack(G, n), zero_cols=5, repeat_cols=[1, 2, 3])
    say("golay + zero/repeated columns")
    run_and_compare(codes.pack(b), b.shape[1], k)


def test_cancel_and_deadline():
    w = WORKLOADS["rand150x75"]
    say("cancel")
    with md.MinDist(w.matrix(), w.n, w.k, cancel_after_chunks=3) as m:
        with pytest.raises(md.MindistError) as e:
            m.run()
        assert e.value.code == -6
        m.set_option("cancel_after_chunks", 0)
        gold = json.load(open(os.path.join(GOLDEN, "rand150x75.json")))
        r = m.run()                           # the context is reusable afterwards
        assert r["d"] == gold["d"]
        compare_with_trace(r, gold["trace"], gold["counts"], gold["pair_min"], None, w.k)
    # the deadline on a code whose run takes about ten times the limit
    # ([255,40], 3e10 codewords of 7 words)
    w = WORKLOADS["rand255x40"]
    say("deadline")
    with md.MinDist(w.matrix(), w.n, w.k, deadline_ms=1) as m:
        with pytest.raises(md.MindistError) as e:
            m.run()
        assert e.value.code == -7
        # a run that stopped with pairs queued leaves nothing behind: the
        # next runs on the context (pairs launched ahead and shared launches
        # reusing its mailboxes) give the full result
        m.set_option("deadline_ms", 0)
        gold = json.load(open(os.path.join(GOLDEN, "rand255x40.json")))
        for _ in range(2):
            r = m.run()
            assert r["d"] == gold["d"]
            compare_with_trace(r, gold["trace"], gold["counts"], gold["pair_min"], None, w.k)


@pytest.mark.parametrize("name", ["rand48x24", "rand150x75"])
def test_injected_upper_bound_must_pass_the_certificate(name):
    """A least weight the device never found (seeded below the true d) makes
    the kernels cut a pair short that the host's own U does not justify: the
    run must fail its certificate with MINDIST_E_CERT; a seed above d changes
    nothing, and the context runs correctly again afterwards."""
    w = WORKLOADS[name]
    G = w.matrix()
    ref = md.min_distance(G, w.n, w.k)
    say("inject U", name, "true d", ref["d"])
    with md.MinDist(G, w.n, w.k, inject_u=ref["d"] - 1) as m:
        with pytest.raises(md.MindistError) as e:
            m.run()
        assert e.value.code == -9
        m.set_option("inject_u", 0)
        r = m.run()
        assert r["d"] == ref["d"]
        check_witness(G, w.n, w.k, r)
    for u in (ref["d"] + 1, ref["d"] + 4):
        r = md.min_distance(G, w.n, w.k, inject_u=u)
        assert r["d"] == ref["d"]
        assert [(p["j"], p["w"], p["pair_min"]) for p in r["pairs"]] == \
               [(p["j"], p["w"], p["pair_min"]) for p in ref["pairs"]]
        check_witness(G, w.n, w.k, r)


def _partial_useful_codes(count):
    """Seeded codes whose partial set reaches the first level its bound term
    is positive (n a little under (m_full + 1) k), with the oracle's
    when-useful run visiting it."""
    rng = PCG32(8080, 11)
    out = []
    while len(out) < count:
        k = rng.uniform_int(4, 24)
        m = rng.uniform_int(1, 3)
        n = m * k + rng.uniform_int(k // 2, k)
        if n <= k or n > 200:
            continue
        G = draw_matrix(rng, n, k)
        try:
            full, part = oracle.partition(G, n, k)
        except oracle.OracleError:
            continue
        r = oracle.bz(G, n, k, partial="when_useful")
        if not any(j == len(full) for j in r["trace"][:, 0].tolist()):
            continue
        out.append((G, n, k))
    return out


def test_partial_set_when_useful_vs_oracle():
    """MINDIST_OPT_PARTIAL = 2: the partial set from the first level its
    bound term is positive, its lower levels caught up then.  Every visited
    pair, bound, minimum and weight sum as the oracle's, under both
    termination rules, on codes that reach that level."""
    for i, (G, n, k) in enumerate(_partial_useful_codes(24)):
        say("partial when useful", i, n, k)
        res, r = run_and_compare(G, n, k, verify=True, partial=2, term=i % 2)
        full, part, _ = md.plan(G, n, k)
        hs = [p["w"] for p in res["pairs"] if p["j"] == len(full)]
        assert hs and hs[0] == 1, hs
        always, _ = run_and_compare(G, n, k, verify=False, partial=0, term=i % 2)
        assert always["d"] == res["d"]


TORCH_STREAM_SCRIPT = r"""
import json, sys
import torch                                  # first: the library then binds to torch's HIP runtime
sys.path.insert(0, sys.argv[1])
import paper_1603_06757_amd as md
from paper_1603_06757_amd.gen import WORKLOADS
w = WORKLOADS["rand150x75"]
s = torch.cuda.Stream()
with torch.cuda.stream(s):
    x = torch.arange(1 << 20, device="cuda", dtype=torch.int64)
    y = x * 3
    with md.MinDist(w.matrix(), w.n, w.k, stream=torch.cuda.current_stream(), verify=1) as m:
        res = m.run()
        z = (y + 1).sum()
s.synchronize()
maps = open("/proc/self/maps").read()
print(json.dumps({"z": int(z.item()), "d": res["d"], "pairs": res["pairs"],
                  "witness": [int(v) for v in res["witness"]], "witness_pair": res["witness_pair"],
                  "witness_rows": res["witness_rows"],
                  "runtimes": sorted({l.split()[-1] for l in maps.splitlines() if "libamdhip64" in l})}))
"""


def test_runs_on_a_torch_stream():
    """MINDIST_OPT_STREAM with torch's current stream: the run's device work
    goes on a stream torch created and owns, ordered with torch work queued
    before and after it on that stream, and the result is the oracle's.
    Torch brings its own HIP runtime, so this runs in a fresh process that
    imports torch before the library (one runtime for both); this process
    loaded the library without torch, and passing it a torch stream raises."""
    import subprocess
    w = WORKLOADS["rand150x75"]
    gold = json.load(open(os.path.join(GOLDEN, "rand150x75.json")))
    G = w.matrix()
    say("rand150x75 on a torch stream (child process)")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, "-c", TORCH_STREAM_SCRIPT, root], capture_output=True,
                       text=True, timeout=240)
    assert p.returncode == 0, p.stderr[-3000:]
    out = json.loads(p.stdout.strip().splitlines()[-1])
    assert len(out["runtimes"]) == 1 and "torch" in out["runtimes"][0], out["runtimes"]
    assert out["z"] == 3 * ((1 << 20) * ((1 << 20) - 1) // 2) + (1 << 20)
    res = {"d": out["d"], "pairs": out["pairs"], "witness": np.array(out["witness"], dtype=np.uint64),
           "witness_pair": tuple(out["witness_pair"]), "witness_rows": out["witness_rows"]}
    assert res["d"] == gold["d"]
    compare_with_trace(res, gold["trace"], gold["counts"], gold["pair_min"], gold["wsum"], w.k)
    check_witness(G, w.n, w.k, res)
    if not md._with_torch:
        with md.MinDist(G, w.n, w.k) as m:
            with pytest.raises(md.MindistError):
                m.set_option("stream", type("S", (), {"cuda_stream": 1})())
