"""CPU pins of the Section 6 code constructions (new linear codes).

The generator matrices are inputs, built from the printed polynomials by
`paper_1603_06757_amd.newcodes`; these checks tie them to what the section
states, with arithmetic of their own (polynomials as Python integers, bit e
= coefficient of x^e):

* f_1 and both f_2 divide x^117 - 1 (so (f_1), (f_2) are cyclic codes of
  length 117 and dimensions 50, 1 and 2); for the [234,52] code (f_2) is
  inside (f_1);
* p is a unit of F_2[x]/(x^117 - 1) (gcd with x^117 - 1 is 1);
* the matrices have the claimed [n, k] and full rank;
* every row is (c, c p mod x^117 - 1) or (0, c) with c in the right cyclic
  code, and the code is closed under the simultaneous cyclic shift of its
  two blocks;
* extension gives even rows; puncturing keeps the dimension (d > 2).
"""
import numpy as np
import pytest

from paper_1603_06757_amd import newcodes as nc

M = 117


def as_int(exps):
    v = 0
    for e in exps:
        v ^= 1 << e
    return v


def row_int(bits):
    v = 0
    for e in np.nonzero(bits)[0]:
        v |= 1 << int(e)
    return v


def pmod(a, b):
    db = b.bit_length() - 1
    while a and a.bit_length() - 1 >= db:
        a ^= b << (a.bit_length() - 1 - db)
    return a


def pmul(a, b):
    out = 0
    while b:
        if b & 1:
            out ^= a
        a <<= 1
        b >>= 1
    return out


def pgcd(a, b):
    while b:
        a, b = b, pmod(a, b)
    return a


X117 = (1 << M) | 1                   # x^117 - 1 = x^117 + 1 over F_2
F2_51 = (1 << 117) - 1              # (x^117 + 1)/(x + 1) = 1 + x + ... + x^116
F2_52 = sum(1 << e for e in range(0, 117, 3)) ^ sum(1 << e for e in range(1, 116, 3))
# (x^117 + 1)/(x^2 + x + 1) = sum over i < 39 of x^(3i) (x + 1): coefficients
# 1 at exponents 0, 1, 3, 4, ..., 114, 115 -- checked below by multiplying back


def rank_gf2(rows):
    """Rank of a list of Python-int rows."""
    basis = {}
    for v in rows:
        while v:
            top = v.bit_length() - 1
            if top in basis:
                v ^= basis[top]
            else:
                basis[top] = v
                break
    return len(basis)


def test_f2_closed_forms():
    assert pmul(F2_51, 0b11) == X117
    assert pmul(F2_52, 0b111) == X117
    assert F2_51.bit_length() - 1 == 116 and F2_52.bit_length() - 1 == 115


def test_f1_generates_a_cyclic_code():
    """f_1 divides x^117 - 1.  (f_2) lies inside (f_1) iff f_1 divides f_2:
    true for the [234,52] code; for the [234,51] code C_2 is the repetition
    code, and the all-ones word is not in (f_1) since x + 1 divides f_1 (it
    has an even number of terms), so those two codes are not nested."""
    f1 = as_int(nc.F1)
    assert f1.bit_length() - 1 == 67
    assert pmod(X117, f1) == 0
    assert pmod(F2_52, f1) == 0
    assert pmod(f1, 0b11) == 0 and pmod(F2_51, f1) != 0


@pytest.mark.parametrize("exps", [nc.P_234_51, nc.P_234_52])
def test_p_is_a_unit(exps):
    p = pmod(as_int(exps), X117)
    assert pgcd(X117, p) == 1


def test_module_polynomial_helpers_agree():
    assert row_int(nc.x_m_minus_1_over((1, 0))) == F2_51
    assert row_int(nc.x_m_minus_1_over((2, 1, 0))) == F2_52
    for exps in (nc.P_234_51, nc.P_234_52):
        assert row_int(nc.reduce_cyclic(nc.poly(exps))) == pmod(as_int(exps), X117)


@pytest.mark.parametrize("k,f2,pexps", [(51, F2_51, nc.P_234_51), (52, F2_52, nc.P_234_52)])
def test_base_code_rows(k, f2, pexps):
    bits = nc.base_code_bits(k)
    assert bits.shape == (k, 2 * M)
    f1 = as_int(nc.F1)
    p = pmod(as_int(pexps), X117)
    rows = [(row_int(b[:M]), row_int(b[M:])) for b in bits]
    for i in range(50):
        c = f1 << i
        assert rows[i] == (c, pmod(pmul(c, p), X117))
    for i in range(k - 50):
        assert rows[50 + i] == (0, f2 << i)
    full = [a | (b << M) for a, b in rows]
    assert rank_gf2(full) == k


@pytest.mark.parametrize("k", [51, 52])
def test_simultaneous_shift_invariance(k):
    bits = nc.base_code_bits(k)
    full = [row_int(b) for b in bits]
    mask = (1 << M) - 1

    def shift(v):
        a, b = v & mask, v >> M
        rot = lambda t: ((t << 1) | (t >> (M - 1))) & mask
        return rot(a) | (rot(b) << M)

    for v in full:
        assert rank_gf2(full + [shift(v)]) == k


@pytest.mark.parametrize("name", sorted(nc.NEW_CODES))
def test_derived_codes(name):
    c = nc.NEW_CODES[name]
    bits = c.bits()
    assert bits.shape == (c.k, c.n)
    assert rank_gf2([row_int(b) for b in bits]) == c.k
    G = c.matrix()
    assert G.shape == (c.k, (c.n + 63) // 64)
    for r in range(c.k):                 # packing: column j at bit j % 64 of word j // 64
        for j in np.nonzero(bits[r])[0][:5]:
            assert (int(G[r, j // 64]) >> (int(j) % 64)) & 1
        assert sum(bin(int(w)).count("1") for w in G[r]) == int(bits[r].sum())
    if c.recipe.startswith("extend"):
        assert (bits.sum(axis=1) % 2 == 0).all()
        src = nc.NEW_CODES[c.recipe.split(":")[1]].bits()
        assert (bits[:, :-1] == src).all()
    if c.recipe.startswith("puncture"):
        _, src, coords = c.recipe.split(":")
        assert c.n == nc.NEW_CODES[src].n - len(coords.split(","))
    assert c.d == c.d_before + 1 or name == "mp235x51" and c.d == c.d_before + 2


def test_extension_chain_and_claims():
    """Section 6's claims fit together: extending the odd-distance [234,51,63]
    gives even distance 64; extending again adds a zero column (every row is
    already even); puncturing lowers the distance by at most one per
    coordinate."""
    c1, c3, c4 = (nc.NEW_CODES[x] for x in ("mp234x51", "mp235x51", "mp236x51"))
    assert c1.d % 2 == 1 and c3.d == c1.d + 1 and c4.d == c3.d
    assert (c4.bits()[:, -1] == 0).all()
    for name, src, drop in (("mp233x51", "mp234x51", 1), ("mp232x51", "mp234x51", 2),
                            ("mp233x52", "mp234x52", 1)):
        assert nc.NEW_CODES[name].d >= nc.NEW_CODES[src].d - drop
