"""The CPU oracle pinned to facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: the pins are textbook weight
enumerators, the plain definition by brute force, closed forms, the paper's
worked examples of lexicographic order and index formulas, and the
stack-based cost lemma (Section 3.3).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1603_06757_amd.gen import random_generator, PCG32, draw_matrix
from tests import codes


def weight_sum_closed_form(Gam, n, k, g):
    """sum over |c| = g of wt(c Gamma) = sum_col sum_{i odd} C(t,i) C(k-t, g-i),
    t = number of rows with a one in that column (a column contributes 1 to
    wt(c Gamma) iff c picks an odd number of its ones)."""
    bits = codes.unpack(Gam, n)
    total = 0
    for col in range(n):
        t = int(bits[:, col].sum())
        total += sum(math.comb(t, i) * math.comb(k - t, g - i) for i in range(1, g + 1, 2))
    return total


# ---- the plain definition on textbook codes --------------------------------

def test_brute_hamming_enumerator():
    G, n, k = codes.hamming7()
    d, dist, wit = oracle.brute(G, n, k)
    assert d == 3
    assert dist.tolist() == [1, 0, 0, 7, 7, 0, 0, 1]


def test_brute_golay_enumerator():
    G, n, k = codes.golay24()
    d, dist, _ = oracle.brute(G, n, k)
    assert d == 8
    want = np.zeros(25, dtype=np.uint64)
    want[[0, 8, 12, 16, 24]] = [1, 759, 2576, 759, 1]
    assert (dist == want).all()


def test_brute_rm15_enumerator():
    G, n, k = codes.reed_muller(1, 5)
    assert (n, k) == (32, 6)
    d, dist, _ = oracle.brute(G, n, k)
    assert d == 16
    assert dist[16] == 62 and dist[32] == 1 and dist.sum() == 64


def test_brute_witness_weight_and_membership():
    G, n, k = codes.golay24()
    d, _, wit = oracle.brute(G, n, k)
    bits = codes.unpack(wit.reshape(1, -1), n)[0]
    assert bits.sum() == d
    # membership: solve for a message over F_2 by brute force on 2^12 messages
    Gb = codes.unpack(G, n)
    msgs = np.array([[(m >> i) & 1 for i in range(k)] for m in range(1 << k)], dtype=np.uint8)
    cw = (msgs @ Gb) % 2
    assert (cw == bits).all(axis=1).any()


def test_brute_rejects_rank_deficient():
    b = np.array([[1, 1, 0, 0], [1, 1, 0, 0]], dtype=np.uint8)
    with pytest.raises(oracle.OracleError):
        oracle.brute(codes.pack(b), 4, 2)


# ---- Brouwer-Zimmerman == plain definition ---------------------------------

@pytest.mark.parametrize("ctor", [codes.hamming7, codes.golay24,
                                  lambda: codes.reed_muller(1, 5),
                                  lambda: codes.reed_muller(1, 4),
                                  lambda: codes.repetition(9),
                                  lambda: codes.even_weight(12)])
def test_bz_textbook_small(ctor):
    G, n, k = ctor()
    d_b, _, _ = oracle.brute(G, n, k)
    for per_level in (False, True):
        for partial in ("always", "never", "when_useful"):
            r = oracle.bz(G, n, k, per_level=per_level, partial=partial)
            assert r["d"] == d_b


def test_bz_equals_brute_random_codes():
    """Plain definition vs Algorithm 1 (both termination rules, the partial
    set always, never or when useful) on 1200 seeded random codes, k <= 20."""
    rng = PCG32(1234, 7)
    checked = 0
    for i in range(1200):
        n = rng.uniform_int(8, 48)
        k = rng.uniform_int(1, min(20, n - 1))
        G = draw_matrix(rng, n, k)
        try:
            d_b, _, _ = oracle.brute(G, n, k)
        except oracle.OracleError:
            continue        # rank deficient draw
        r = oracle.bz(G, n, k)
        assert r["d"] == d_b, (i, n, k)
        rl = oracle.bz(G, n, k, per_level=True)
        assert rl["d"] == d_b
        rn = oracle.bz(G, n, k, partial_never=True)
        assert rn["d"] == d_b
        ru = oracle.bz(G, n, k, partial="when_useful")
        assert ru["d"] == d_b
        checked += 1
    assert checked > 1000


def test_bz_equals_brute_k20():
    for seed in range(6):
        G = random_generator(44, 20, 99, seed)
        d_b, _, _ = oracle.brute(G, 44, 20)
        assert oracle.bz(G, 44, 20)["d"] == d_b


def test_bz_workload_48x24_brute():
    G = random_generator(48, 24, 1, 0, 0)
    d_b, dist, _ = oracle.brute(G, 48, 24)
    r = oracle.bz(G, 48, 24, threads=4)
    assert r["d"] == d_b
    assert r["m_full"] == 2 and r["k_m"] == 0


@pytest.mark.parametrize("r_,m_,d_", [(2, 6, 16), (2, 7, 32)])
def test_bz_reed_muller_large_k(r_, m_, d_):
    G, n, k = codes.reed_muller(r_, m_)
    res = oracle.bz(G, n, k, threads=8)
    assert res["d"] == d_


def test_bz_punctured_rm(tmp_path):
    G, n, k = codes.reed_muller(1, 6, puncture_last=True)   # [63,7,31]
    d_b, _, _ = oracle.brute(G, n, k)
    assert d_b == 31
    assert oracle.bz(G, n, k)["d"] == 31


def test_bz_zero_and_repeated_columns():
    G, n, k = codes.golay24()
    b = codes.with_extra_columns(codes.unpack(G, n), zero_cols=3)
    assert oracle.bz(codes.pack(b), b.shape[1], k)["d"] == 8
    b2 = codes.with_extra_columns(codes.unpack(G, n), repeat_cols=[0, 1, 2, 3])
    d_b, _, _ = oracle.brute(codes.pack(b2), b2.shape[1], k)
    assert oracle.bz(codes.pack(b2), b2.shape[1], k)["d"] == d_b


def test_bz_witness_certificate():
    G = random_generator(60, 20, 5, 3)
    r = oracle.bz(G, 60, 20)
    bits = codes.unpack(r["witness"].reshape(1, -1), 60)[0]
    assert bits.sum() == r["d"]
    # witness lies in the row space: rank of [G; x] stays k
    Gb = codes.unpack(G, 60)
    assert _rank(np.vstack([Gb, bits])) == 20
    # it is the XOR of the recorded rows of the recorded Gamma_j
    j, g = r["witness_pair"]
    assert len(r["witness_combo"]) == g


def _rank(bits):
    M = bits.copy() % 2
    r = 0
    for c in range(M.shape[1]):
        piv = [i for i in range(r, M.shape[0]) if M[i, c]]
        if not piv:
            continue
        M[[r, piv[0]]] = M[[piv[0], r]]
        for i in range(M.shape[0]):
            if i != r and M[i, c]:
                M[i] ^= M[r]
        r += 1
    return r


# ---- information sets and systematic matrices -------------------------------

def test_partition_hand_example():
    # columns: 0,1 independent; 2 = 0; 3 = 1; 4 = 0+1; 5 zero
    b = np.array([[1, 0, 1, 0, 1, 0],
                  [0, 1, 0, 1, 1, 0]], dtype=np.uint8)
    full, part = oracle.partition(codes.pack(b), 6, 2)
    assert full == [[0, 1], [2, 3]]
    assert part == [4]          # rank 1 left over; the zero column adds nothing


def test_partition_invariants_random():
    for seed in range(20):
        n, k = 90, 25
        G = random_generator(n, k, 77, seed)
        full, part = oracle.partition(G, n, k)
        cols = [c for s in full for c in s] + part
        assert len(cols) == len(set(cols))
        for s in full:
            assert s == sorted(s) and len(s) == k
            assert _rank(codes.unpack(G, n)[:, s]) == k
        assert part == sorted(part)
        left = sorted(set(range(n)) - {c for s in full for c in s})
        assert _rank(codes.unpack(G, n)[:, left]) == len(part) if left else part == []


def test_gamma_is_systematic_and_row_equivalent():
    n, k = 70, 30
    G = random_generator(n, k, 11, 0)
    full, part = oracle.partition(G, n, k)
    Gb = codes.unpack(G, n)
    for s in full:
        Gam = codes.unpack(oracle.gamma(G, n, k, s), n)
        assert (Gam[:, s] == np.eye(k, dtype=np.uint8)).all()
        assert _rank(np.vstack([Gb, Gam])) == k
    if part:
        Gam = codes.unpack(oracle.gamma(G, n, k, part), n)
        km = len(part)
        assert (Gam[:km, part] == np.eye(km, dtype=np.uint8)).all()
        assert (Gam[km:, part] == 0).all()
        assert _rank(np.vstack([Gb, Gam])) == k


def _assert_rref(Gam, order, first):
    """Reduced row echelon form under a column order, by its definition: the
    leading one of each row (first nonzero in that order) lies strictly to
    the right of the one above, every leading column is a unit vector, and
    the first len(first) leading columns are the set's own columns."""
    k = Gam.shape[0]
    pos = {c: i for i, c in enumerate(order)}
    lead = []
    for r in range(k):
        nz = [c for c in order if Gam[r, c]]
        assert nz, f"row {r} is zero"
        lead.append(nz[0])
    assert all(pos[lead[r]] < pos[lead[r + 1]] for r in range(k - 1))
    for r, c in enumerate(lead):
        col = np.zeros(k, dtype=np.uint8)
        col[r] = 1
        assert (Gam[:, c] == col).all(), f"pivot column {c} of row {r} is not a unit vector"
    assert lead[:len(first)] == list(first)
    return lead


def test_gamma_is_the_reduced_echelon_form_partial_set_included():
    """Section 2's [[I, A], [0, B]] form of the partial set made unique: every
    Gamma_j is the reduced row echelon form of G under (set columns, then the
    others ascending), so the lower block's pivots lie outside the set,
    ascend, and are cleared in the upper rows too."""
    seen_lower = 0
    for (n, k, seed) in [(70, 30, 0), (100, 30, 9), (110, 24, 3), (90, 25, 4)]:
        G = random_generator(n, k, 11 if n == 70 else seed, 0)
        full, part = oracle.partition(G, n, k)
        Gb = codes.unpack(G, n)
        for s in full + ([part] if part else []):
            order = list(s) + [c for c in range(n) if c not in set(s)]
            Gam = codes.unpack(oracle.gamma(G, n, k, s), n)
            lead = _assert_rref(Gam, order, s)
            assert _rank(np.vstack([Gb, Gam])) == k
            lower = lead[len(s):]
            assert all(c not in set(s) for c in lower) and lower == sorted(lower)
            seen_lower += len(lower)
    assert seen_lower > 0


# ---- enumeration of one pair ------------------------------------------------

def test_lexicographic_order_example():
    """Section 3.2: for 50 choose 3 the order is (0,1,2),(0,1,3),...,(0,1,49),(0,2,3),..."""
    Gam = np.eye(50, dtype=np.uint8)
    P = codes.pack(np.concatenate([Gam, np.zeros((50, 1), np.uint8)], axis=1))
    first = [oracle.combo_codeword(P, 51, 50, 3, r)[0] for r in range(49)]
    assert first[0] == [0, 1, 2] and first[1] == [0, 1, 3] and first[47] == [0, 1, 49]
    assert first[48] == [0, 2, 3]


def test_index_of_worked_examples():
    """Section 3.4: with k=50, a=3, b=2 the first left combination not to be
    processed has index C(50,3) - C(4,3) = 19596, i.e. (46,47,48); the first
    right combination for last-left 47 has index C(50,2) - C(2,2) = 1224,
    i.e. (48,49)."""
    P = codes.pack(np.concatenate([np.eye(50, dtype=np.uint8), np.zeros((50, 1), np.uint8)], axis=1))
    assert oracle.combo_codeword(P, 51, 50, 3, 19596)[0] == [46, 47, 48]
    assert oracle.combo_codeword(P, 51, 50, 3, 19599)[0] == [47, 48, 49]
    assert oracle.combo_codeword(P, 51, 50, 2, 1224)[0] == [48, 49]


@pytest.mark.parametrize("k,g", [(6, 3), (8, 4), (10, 5), (9, 2), (12, 6), (20, 4)])
def test_stack_cost_lemma(k, g):
    """Section 3.3 lemma: C(k,g)+C(k-1,g-1)+...+C(k-g+2,2) row additions."""
    Gam = random_generator(40, k, 3, k)
    _, _, _, cnt, adds = oracle.pair(Gam, 40, k, g)
    assert cnt == math.comb(k, g)
    assert adds == sum(math.comb(k - i, g - i) for i in range(0, g - 1))


@pytest.mark.parametrize("n,k,g", [(150, 75, 1), (150, 75, 2), (150, 75, 3),
                                   (255, 40, 4), (48, 24, 6), (100, 30, 5)])
def test_pair_weight_sum_closed_form(n, k, g):
    G = random_generator(n, k, 21, n + g)
    full, _ = oracle.partition(G, n, k)
    Gam = oracle.gamma(G, n, k, full[0])
    m, _, ws, cnt, _ = oracle.pair(Gam, n, k, g, threads=4)
    assert cnt == math.comb(k, g)
    assert ws == weight_sum_closed_form(Gam, n, k, g)


def test_pair_ranges_partition_the_pair():
    n, k, g = 80, 30, 4
    G = random_generator(n, k, 8, 1)
    Gam = oracle.gamma(G, n, k, oracle.partition(G, n, k)[0][0])
    whole = oracle.pair(Gam, n, k, g)
    tot = math.comb(k, g)
    cuts = [0, 1, 777, 5000, tot - 3, tot]
    mins, sums, cnts = [], 0, 0
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        m, _, ws, cnt, _ = oracle.pair(Gam, n, k, g, lo, hi)
        mins.append(m)
        sums += ws
        cnts += cnt
    assert min(mins) == whole[0] and sums == whole[2] and cnts == tot


def test_every_gamma_enumerates_the_whole_code():
    """For each Gamma_j, the pairs over all levels cover every nonzero
    codeword once: the weight sums add up to sum_w w A_w of the brute force."""
    G, n, k = codes.golay24()
    _, dist, _ = oracle.brute(G, n, k)
    target = sum(w * int(a) for w, a in enumerate(dist))
    full, part = oracle.partition(G, n, k)
    for s in full + ([part] if part else []):
        Gam = oracle.gamma(G, n, k, s)
        assert sum(oracle.pair(Gam, n, k, g)[2] for g in range(1, k + 1)) == target


# ---- Algorithm 1 control -----------------------------------------------------

def test_bz_counts_are_binomials_and_bound_sound():
    G = random_generator(48, 24, 1, 0, 0)
    r = oracle.bz(G, 48, 24)
    for (j, g, Lb, La, U, pm) in r["trace"].tolist():
        assert r["counts"][j, g] == math.comb(24, g)
        assert r["pair_min"][j, g] == pm
        assert pm >= Lb            # nothing below the bound before the pair
    assert r["L_final"] >= r["d"]


def test_bz_per_level_visits_whole_levels():
    G = random_generator(48, 24, 1, 0, 0)
    r = oracle.bz(G, 48, 24, per_level=True)
    gs = r["trace"][:, 1].tolist()
    for g in set(gs):
        assert gs.count(g) == r["n_gamma"]


def test_generator_matches_published_pcg32_demo():
    rng = PCG32(42, 54)
    assert [rng.next_u32() for _ in range(6)] == [
        0xa15c02b7, 0x7b47f409, 0xba1d3330, 0x83d2f293, 0xbfa4784b, 0xcbed606e]


def test_bz_per_level_bound_is_the_printed_formula():
    """Algorithm 1: after level g, L = (m-1)(g+1) + max(0, g+1-k+k_m), with
    m-1 full sets and a partial set of rank k_m (term 0 without one)."""
    for (n, k, seed) in [(110, 24, 3), (100, 30, 9), (48, 24, 1)]:
        G = random_generator(n, k, seed, 0)
        r = oracle.bz(G, n, k, per_level=True)
        mf, km = r["m_full"], r["k_m"]
        g = r["last_level"]
        part = max(0, g + 1 - k + km) if km >= 1 else 0
        assert r["L_final"] == mf * (g + 1) + part


def test_bz_per_pair_matches_printed_formula_at_level_ends():
    """Raising L after every Gamma_j ends each level at the printed value."""
    for (n, k, seed) in [(110, 24, 3), (100, 30, 9)]:
        G = random_generator(n, k, seed, 0)
        r = oracle.bz(G, n, k)
        mf, km, ng = r["m_full"], r["k_m"], r["n_gamma"]
        assert km >= 1
        for (j, g, Lb, La, U, pm) in r["trace"].tolist():
            if j == ng - 1:
                assert La == mf * (g + 1) + max(0, g + 1 - k + km)
            if j == 0 and g > 1:
                assert Lb == mf * g + max(0, g - k + km)


# ---- the lower bound is a lower bound ------------------------------------------

def _all_codewords(Gb):
    k = Gb.shape[0]
    msgs = ((np.arange(1 << k)[:, None] >> np.arange(k)[None, :]) & 1).astype(np.uint8)
    return ((msgs @ Gb) % 2)[1:]


def _assert_bound_sound(G, n, k, **kw):
    """Section 2's lower bound by its meaning: after each visited pair, every
    nonzero codeword that no pair (j, h) so far has enumerated -- its message
    under Gamma_j, read at the pivot columns, does not weigh h -- weighs at
    least L (brute force over all 2^k codewords)."""
    r = oracle.bz(G, n, k, **kw)
    full, part = oracle.partition(G, n, k)
    sets = full + ([part] if part and r["n_gamma"] > len(full) else [])
    X = _all_codewords(codes.unpack(G, n))
    wt = X.sum(axis=1)
    msg_wt = []
    for s in sets:
        order = list(s) + [c for c in range(n) if c not in set(s)]
        lead = _assert_rref(codes.unpack(oracle.gamma(G, n, k, s), n), order, s)
        msg_wt.append(X[:, lead].sum(axis=1))
    covered = np.zeros(len(X), dtype=bool)
    for (j, h, Lb, La, U, pm) in r["trace"].tolist():
        left = wt[~covered]
        assert left.size == 0 or left.min() >= Lb, (j, h, "before", Lb, left.min())
        covered |= msg_wt[j] == h
        left = wt[~covered]
        assert left.size == 0 or left.min() >= La, (j, h, "after", La, left.min())
    return r


def test_lower_bound_is_sound_by_brute_force():
    """Every rule and partial-set policy, on 300 seeded random codes with
    k <= 13: no codeword left unenumerated weighs less than L."""
    rng = PCG32(4321, 9)
    checked = 0
    for _ in range(300):
        n = rng.uniform_int(10, 40)
        k = rng.uniform_int(4, min(13, n - 1))
        G = draw_matrix(rng, n, k)
        try:
            oracle.brute(G, n, k)
        except oracle.OracleError:
            continue
        for kw in ({}, {"per_level": True}, {"partial": "when_useful"},
                   {"partial": "when_useful", "per_level": True}, {"partial": "never"}):
            _assert_bound_sound(G, n, k, **kw)
        checked += 1
    assert checked > 250


def _when_useful_code():
    """A [27,6] code whose partial set (rank 4, so its bound term is positive
    from level 2 on) holds the only codeword of weight 6 at message weight 1:
    x = (1,1,1,0,0,0) G weighs 3 on each full set and vanishes on the 15
    remaining columns, which span only the 4 functionals orthogonal to
    (1,1,1,0,0,0) and (0,0,0,1,1,1)."""
    k = 6
    B = np.array([[1, 1, 1, 0, 1, 1], [1, 0, 0, 1, 0, 0], [0, 1, 0, 1, 0, 0],
                  [1, 1, 1, 1, 0, 0], [1, 1, 1, 0, 0, 1], [0, 0, 1, 0, 1, 0]], dtype=np.uint8)
    perp = np.array([[1, 1, 0, 0, 0, 0], [1, 0, 1, 0, 0, 0],
                     [0, 0, 0, 1, 1, 0], [0, 0, 0, 1, 0, 1]], dtype=np.uint8).T
    pats = np.array([[(v >> b) & 1 for b in range(4)] for v in range(1, 16)], dtype=np.uint8).T
    bits = np.concatenate([np.eye(k, dtype=np.uint8), B, (perp @ pats) % 2], axis=1)
    return codes.pack(bits), bits.shape[1], k


def test_partial_set_when_useful_catches_up_its_lower_levels():
    """Deferring the partial set to its first useful level: its bound term
    at level 2 needs the set's level 1 too.  Here that level holds the only
    codeword of minimum weight, found by the catch-up pair (2, 1)."""
    G, n, k = _when_useful_code()
    d, _, _ = oracle.brute(G, n, k)
    assert d == 6
    full, part = oracle.partition(G, n, k)
    assert len(full) == 2 and len(part) == 4
    r = _assert_bound_sound(G, n, k, partial="when_useful")
    assert r["d"] == 6
    assert [tuple(t[:2]) for t in r["trace"].tolist()] == [(0, 1), (1, 1), (0, 2), (1, 2), (2, 1)]
    assert r["witness_pair"] == (2, 1)
    for policy in ("always", "never"):
        assert oracle.bz(G, n, k, partial=policy)["d"] == 6


# ---- the pins catch plausible mistakes ----------------------------------------

def _fails(pin):
    try:
        pin()
    except (AssertionError, oracle.OracleError):
        return True
    return False


# planted mistake -> pins expected to catch it (see the list in mindist_oracle.c)
_CATCHERS = {
    1: [test_bz_per_level_bound_is_the_printed_formula,
        test_bz_per_pair_matches_printed_formula_at_level_ends],
    2: [test_bz_equals_brute_random_codes, test_bz_equals_brute_k20,
        test_lower_bound_is_sound_by_brute_force],
    3: [lambda: test_stack_cost_lemma(8, 4), lambda: test_pair_weight_sum_closed_form(100, 30, 5),
        test_bz_counts_are_binomials_and_bound_sound],
    4: [test_gamma_is_systematic_and_row_equivalent],
    6: [test_gamma_is_the_reduced_echelon_form_partial_set_included],
    7: [test_partial_set_when_useful_catches_up_its_lower_levels],
    5: [lambda: test_pair_weight_sum_closed_form(150, 75, 2),
        lambda: test_bz_reed_muller_large_k(2, 7, 32)],
}


@pytest.mark.parametrize("fault", sorted(_CATCHERS))
def test_planted_mistakes_are_caught(fault):
    """Each planted mistake (a dropped bound term, a wrong level index, a
    skipped combination, an incomplete reduction, a dropped word, a partial
    set whose lower block is left unreduced above its pivots, a deferred
    partial set counted without its lower levels) makes at
    least one pin fail; with no mistake planted all of them pass."""
    with oracle.planted(fault):
        caught = [_fails(p) for p in _CATCHERS[fault]]
    assert any(caught), f"mistake {fault} passed every pin"
    assert not any(_fails(p) for p in _CATCHERS[fault])
