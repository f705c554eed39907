"""Host logic of the HIP library, checked on the CPU (no device needed).

The library's partition and systematic matrices are an independent
implementation (row Gauss-Jordan sweeps) of the same canonical readings the
oracle follows (column XOR basis + a separate echelon form); they must agree
bit for bit.  Also: the C ABI loads and exports every declared entry point.
"""
import ctypes
import itertools
import math
import os
import re

import numpy as np
import pytest

import oracle
import paper_1603_06757_amd as md
from paper_1603_06757_amd.gen import WORKLOADS, random_generator, batch_code
from tests import codes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols(header="mindist.h"):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mindist_[a-z_0-9]+)\s*\(", text)))


def test_cpu_library_exports_its_symbols_and_stays_separate():
    """libmindist_cpu.so (the paper's CPU algorithms) exports what
    mindist_cpu.h declares; the GPU library holds none of it."""
    from paper_1603_06757_amd import cpu
    syms = declared_symbols("mindist_cpu.h")
    assert syms == ["mindist_cpu_pair"]
    L = ctypes.CDLL(cpu.LIB_PATH)
    for s in syms:
        assert hasattr(L, s), s
    assert not hasattr(ctypes.CDLL(md.LIB_PATH), "mindist_cpu_pair")


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(md.LIB_PATH)
    syms = declared_symbols()
    assert "mindist_create" in syms and "mindist_run" in syms
    assert "mindist_run_batch" in syms and "mindist_server_submit" in syms
    for s in syms:
        assert hasattr(L, s), s


def _cases():
    out = [codes.hamming7(), codes.golay24(), codes.reed_muller(1, 5), codes.reed_muller(2, 7),
           codes.reed_muller(2, 8), codes.repetition(7), codes.even_weight(10)]
    for w in WORKLOADS.values():
        out.append((w.matrix(), w.n, w.k))
    for i in range(40):
        n, k, G = batch_code(i)
        out.append((G, n, k))
    for s in range(20):
        out.append((random_generator(100, 33, 404, s), 100, 33))
    return out


def test_plan_matches_oracle_bit_for_bit():
    for G, n, k in _cases():
        full, part, gam = md.plan(G, n, k)
        ofull, opart = oracle.partition(G, n, k)
        assert full == ofull and part == opart, (n, k)
        sets = full + ([part] if part else [])
        assert gam.shape[0] == len(sets)
        for j, s in enumerate(sets):
            assert (gam[j] == oracle.gamma(G, n, k, s)).all(), (n, k, j)


def test_plan_errors():
    G, n, k = codes.hamming7()
    bad = G.copy()
    bad[0, 0] |= np.uint64(1) << np.uint64(7)   # bit beyond column n-1
    with pytest.raises(md.MindistError) as e:
        md.plan(bad, n, k)
    assert e.value.code == -1
    dep = codes.pack(np.array([[1, 0, 1, 1], [1, 0, 1, 1]], dtype=np.uint8))
    with pytest.raises(md.MindistError) as e:
        md.plan(dep, 4, 2)
    assert e.value.code == -2
    with pytest.raises(md.MindistError):
        md.plan(np.zeros((3, 1), np.uint64), 3, 3)        # n must exceed k


def test_bound_schedule_matches_printed_formula_at_level_ends():
    """Per-Gamma bounds end each level at Algorithm 1's value
    (m-1)(g+1) + max(0, g+1-k+k_m), and start a level at its value for g-1."""
    for (k, mf, km) in [(40, 6, 15), (75, 2, 0), (24, 2, 0), (30, 3, 10), (37, 6, 34)]:
        ng = mf + (1 if km >= 1 else 0)
        for g in range(1, 12):
            end = md.bound_after(k, mf, km, 1, ng - 1, g)
            assert end == mf * (g + 1) + (max(0, g + 1 - k + km) if km >= 1 else 0)
            for j in range(ng):
                v = md.bound_after(k, mf, km, 1, j, g)
                assert v >= (mf * g + (max(0, g - k + km) if km >= 1 else 0))
                assert v <= end


def test_bound_rejects_bad_queries():
    with pytest.raises(md.MindistError):
        md.bound_after(40, 6, 15, 1, 7, 3)


def test_binding_structs_match_the_c_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    the C compiler gives the header's struct (a mismatch would corrupt every
    result silently)."""
    import shutil
    import subprocess
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    pairs = [("mindist_result", md.Result), ("mindist_pair", md.Pair),
             ("mindist_batch_opts", md.BatchOpts), ("mindist_server_opts", md.ServerOpts),
             ("mindist_server_result", md.ServerResult), ("mindist_server_stats", md.ServerStats)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mindist.h"', "int main(void) {"]
    for cname, py in pairs:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "abi"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, f, v = line.split()
        got[(cname, f)] = int(v)
    for cname, py in pairs:
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_server_rejects_an_unknown_engine():
    """Argument checks of mindist_server_create run before any device call."""
    with pytest.raises(md.MindistError) as e:
        md.Server(engine=2)
    assert e.value.code == -1


def _colex_key(c):
    return tuple(reversed(c))


def test_colex_unrank_is_the_colex_bijection():
    """Every rank of every (hi, r) with hi <= 14, and (hi, r) up to 20 where
    C(hi, r) <= 20000: the subsets come out ascending, distinct, in colex
    order (so rank + 1 is the colex successor), with sum_t C(x_t, t) = rank
    (t from 1) -- against itertools' enumeration sorted by the colex key."""
    for hi in range(0, 21):
        for r in range(0, hi + 1):
            total = math.comb(hi, r)
            if hi > 14 and total > 20000:
                continue
            want = sorted(itertools.combinations(range(hi), r), key=_colex_key)
            got = [tuple(md.colex_unrank(i, r, hi)) for i in range(total)]
            assert got == want, (hi, r)
            for i in (0, total - 1):
                assert sum(math.comb(x, t + 1) for t, x in enumerate(got[i])) == i


def test_colex_unrank_rejects_bad_queries():
    for rank, r, hi in ((10, 2, 5), (0, 3, 2), (0, 65, 512), (0, 2, 513)):
        with pytest.raises(md.MindistError) as e:
            md.colex_unrank(rank, r, hi)
        assert e.value.code == -1


def test_option_and_error_codes_match_the_header():
    text = open(os.path.join(ROOT, "include", "mindist.h")).read()
    opts = {m.group(1).lower(): int(m.group(2))
            for m in re.finditer(r"#define MINDIST_OPT_(\w+)\s+(\d+)", text)}
    errs = {int(m.group(2)): "E_" + m.group(1)
            for m in re.finditer(r"#define MINDIST_E_(\w+)\s+(-\d+)", text)}
    assert opts == md.OPT
    assert {k: v for k, v in md.E_NAMES.items() if k < 0} == errs


# ---- Algorithm 1's pair order and the run certificate (host-only) ----------

def _policy_cases():
    """Seeded random codes whose partial sets reach their first useful level
    (n a little under (m_full + 1) k), plus the workloads' shapes."""
    from paper_1603_06757_amd.gen import PCG32, draw_matrix
    rng = PCG32(4321, 3)
    out = []
    while len(out) < 60:
        k = rng.uniform_int(3, 14)
        m = rng.uniform_int(1, 3)
        n = min(m * k + rng.uniform_int(1, k), 80)
        if n <= k:
            continue
        G = draw_matrix(rng, n, k)
        try:
            oracle.partition(G, n, k)
        except oracle.OracleError:
            continue
        out.append((G, n, k))
    return out


POLICY_VARIANTS = [("always", False), ("always", True), ("never", False), ("never", True),
                   ("when_useful", False), ("when_useful", True)]


def test_schedule_matches_the_oracles_visiting_order():
    """The library's pair order and bounds (mindist_schedule) against the
    oracle's visited pairs under every partial-set policy and termination
    rule: the oracle's trace is a prefix of the schedule, with the same L
    after every pair."""
    reached = 0
    for G, n, k in _policy_cases():
        full, part = oracle.partition(G, n, k)
        for partial, per_level in POLICY_VARIANTS:
            r = oracle.bz(G, n, k, partial=partial, per_level=per_level)
            sched = md.schedule(k, len(full), len(part), partial, per_level)
            tr = r["trace"].tolist()
            assert len(tr) <= len(sched)
            for (j, h, Lb, La, U, pm), (sj, sh, sg, sL) in zip(tr, sched):
                assert (j, h, La) == (sj, sh, sL), (n, k, partial, per_level)
            if partial == "when_useful" and any(j == len(full) for j, *_ in tr):
                reached += 1
    assert reached >= 5


def _records(r, k):
    """The oracle's trace as the library's pair records (every pair complete)."""
    return [{"j": j, "w": h, "L_before": Lb, "L_after": La, "U_after": U, "pair_min": pm,
             "count": math.comb(k, h), "executed": math.comb(k, h)}
            for j, h, Lb, La, U, pm in r["trace"].tolist()]


def _certify(r, n, k, recs, d=None, L_final=None, exited=0, **kw):
    return md.certify(n, k, r["m_full"], r["k_m"], recs, r["d"] if d is None else d,
                      r["L_final"] if L_final is None else L_final, exited, **kw)


def test_certificate_accepts_the_oracles_runs():
    for G, n, k in _policy_cases()[:30]:
        for partial, per_level in POLICY_VARIANTS:
            r = oracle.bz(G, n, k, partial=partial, per_level=per_level)
            assert _certify(r, n, k, _records(r, k), partial=partial, per_level=per_level) == 0


def _expect_cert(fn):
    with pytest.raises(md.MindistError) as e:
        fn()
    assert e.value.code == -9, e.value


def test_certificate_rejects_broken_traces():
    """Synthetic pair records: each plausible fault of a device sequencer or
    a host loop ends in MINDIST_E_CERT."""
    w = WORKLOADS["rand48x24"]
    G, n, k = w.matrix(), w.n, w.k
    r = oracle.bz(G, n, k)
    base = _records(r, k)
    assert len(base) >= 3
    assert _certify(r, n, k, base) == 0

    def mutated(t, **kv):
        recs = [dict(p) for p in base]
        recs[t].update(kv)
        return recs
    # a completed pair that evaluated fewer or more combinations than C(k,w)
    _expect_cert(lambda: _certify(r, n, k, mutated(0, executed=base[0]["count"] - 1)))
    _expect_cert(lambda: _certify(r, n, k, mutated(1, executed=base[1]["count"] + 1)))
    # a wrong count, a wrong bound, a wrong U
    _expect_cert(lambda: _certify(r, n, k, mutated(1, count=base[1]["count"] + 1)))
    _expect_cert(lambda: _certify(r, n, k, mutated(1, L_after=base[1]["L_after"] + 1)))
    _expect_cert(lambda: _certify(r, n, k, mutated(2, L_before=base[2]["L_before"] - 1)))
    _expect_cert(lambda: _certify(r, n, k, mutated(0, U_after=base[0]["U_after"] - 1)))
    # pairs out of order, a pair dropped, the run stopped early
    sw = [dict(p) for p in base]
    sw[0]["j"], sw[1]["j"] = sw[1]["j"], sw[0]["j"]
    _expect_cert(lambda: _certify(r, n, k, sw))
    _expect_cert(lambda: _certify(r, n, k, base[:1] + base[2:]))
    short = base[:-1]
    _expect_cert(lambda: _certify(r, n, k, short, L_final=short[-1]["L_after"]))
    # a pair visited after L >= U
    extra = dict(base[-1])
    _expect_cert(lambda: _certify(r, n, k, base + [extra]))
    # d or the final bound misreported
    _expect_cert(lambda: _certify(r, n, k, base, d=r["d"] - 1))
    _expect_cert(lambda: _certify(r, n, k, base, L_final=r["L_final"] + 1))
    # a cut last pair: justified only when U <= L before it, and only last
    last = dict(base[-1], executed=base[-1]["count"] // 2, L_after=base[-1]["L_before"])
    cut = base[:-1] + [last]
    U_before_last = cut[-1]["U_after"]
    if U_before_last <= last["L_before"]:
        assert _certify(r, n, k, cut, L_final=last["L_before"], exited=1) == 0
        _expect_cert(lambda: _certify(r, n, k, cut, L_final=last["L_before"], exited=0))
        _expect_cert(lambda: _certify(r, n, k, cut, L_final=last["L_before"], exited=1,
                                      midpair_exit=False))
    mid = mutated(0, executed=base[0]["count"] // 2)
    _expect_cert(lambda: _certify(r, n, k, mid, exited=1))


def test_certificate_rejects_an_unjustified_cut():
    """A pair cut short while the least weight found is above the bound
    before it (what a least weight the device never found would cause)."""
    w = WORKLOADS["rand48x24"]
    G, n, k = w.matrix(), w.n, w.k
    r = oracle.bz(G, n, k)
    base = _records(r, k)
    t = 1
    assert base[t]["U_after"] > base[t]["L_before"]
    recs = base[:t] + [dict(base[t], executed=5, L_after=base[t]["L_before"])]
    _expect_cert(lambda: _certify(r, n, k, recs, d=recs[-1]["U_after"],
                                  L_final=base[t]["L_before"], exited=1))


def test_pair_records_convert_to_the_same_dicts():
    """The binding's numpy view of pair records gives exactly the dicts of
    the ctypes fields (types included), for every field of the struct."""
    import random
    arr = (md.Pair * 40)()
    rng = random.Random(3)
    for i in range(40):
        p = arr[i]
        for f, t in md.Pair._fields_:
            if t is ctypes.c_int32:
                setattr(p, f, rng.randint(-2**31, 2**31 - 1))
            elif t is ctypes.c_uint64:
                setattr(p, f, rng.randint(0, 2**64 - 1))
            else:
                setattr(p, f, rng.random() * 1e6)
    ref = [arr[i].to_dict() for i in range(40)]
    got = md._pair_dicts(arr, 0, 40)
    assert got == ref
    assert [type(v) for v in got[0].values()] == [type(v) for v in ref[0].values()]
    assert md._pair_dicts(arr, 7, 19) == ref[7:19]
    assert md._pair_dicts(arr, 5, 5) == []


def _bit_bytes4(x, c):
    # the kernel's expansion: bits 4c..4c+3 of x as bytes 0/1 (one 24-bit
    # multiply spreads a nibble over four bytes, the mask keeps bit 0 of each)
    return ((((x >> (4 * c)) & 0xF) * 0x00204081) & 0xFFFFFFFF) & 0x01010101


def _bytes16(x, pm):
    """16 low bits of x as 16 int8 values, as the kernel builds an operand:
    0/1 (pm False) or +1 for a clear bit / -1 for a set bit (pm True)."""
    out = []
    for c in range(4):
        b = _bit_bytes4(x, c)
        if pm:
            b = ((((b << 8) - b) & 0xFFFFFFFF) | 0x01010101)
        out += [((b >> (8 * p)) & 0xFF) for p in range(4)]
    return np.array(out, dtype=np.uint8).view(np.int8).astype(np.int64)


def test_matrix_core_operand_bytes():
    """Every nibble expands to its bits, one byte each; the +-1 form is 1 - 2 bit."""
    for x in range(1 << 16):
        if x % 97 and x not in (0, 0xFFFF):
            continue
        bits = np.array([(x >> p) & 1 for p in range(16)], dtype=np.int64)
        assert (_bytes16(x, False) == bits).all()
        assert (_bytes16(x, True) == 1 - 2 * bits).all()


def test_matrix_core_block_is_the_weights():
    """One 32 x 32 block as the matrix-core loop computes it -- lane i + 32h
    holds bits 16h..16h+15 of each word of row (right sum) or column (left
    sum) i, D products of 32 bytes summed per (row, column), plus wt(l) --
    equals popcount(l ^ r) for every pair (wt(l ^ r) = wt(l) + sum_k r_k
    (1 - 2 l_k)).  The lane layout is the one a one-wave probe of
    v_mfma_i32_32x32x32_i8 showed on the GPU; here it is only taken as given."""
    rng = np.random.default_rng(1603)
    for D in (1, 2, 3, 4):
        for trial in range(3):
            R = rng.integers(0, 1 << 32, size=(32, D), dtype=np.uint64)
            Lf = rng.integers(0, 1 << 32, size=(32, D), dtype=np.uint64)
            if trial == 1:       # the top word partly used, as in n - k = 75
                R[:, -1] &= 0x7FF
                Lf[:, -1] &= 0x7FF
            acc = np.zeros((32, 32), dtype=np.int64)
            for d in range(D):
                A = np.zeros((64, 16), dtype=np.int64)
                Bm = np.zeros((64, 16), dtype=np.int64)
                for lane in range(64):
                    i, h = lane % 32, lane // 32
                    A[lane] = _bytes16(int(R[i, d]) >> (16 * h), False)
                    Bm[lane] = _bytes16(int(Lf[i, d]) >> (16 * h), True)
                # D[i][j] = sum_h sum_p A[i + 32h][p] * B[j + 32h][p]
                acc += A[:32] @ Bm[:32].T + A[32:] @ Bm[32:].T
            for i in range(32):
                for j in range(32):
                    wl = sum(bin(int(Lf[j, d])).count("1") for d in range(D))
                    want = sum(bin(int(R[i, d]) ^ int(Lf[j, d])).count("1") for d in range(D))
                    assert wl + acc[i, j] == want
