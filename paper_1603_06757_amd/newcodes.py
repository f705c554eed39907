"""The codes of Section 6 (new linear codes), built from their printed data.

A matrix-product code with polynomial units is C = [C_1 C_2] . A with
A = [[1, p], [0, 1]] over R = F_2[x]/(x^m - 1): its codewords are
(c_1, c_1 p + c_2) for c_1 in C_1 and c_2 in C_2, two blocks of m
coordinates.  C_1 = (f_1) and C_2 = (f_2) are cyclic codes of length
m = 117; the section prints f_1, f_2 and the unit p for the two base codes
[234,51,63] and [234,52,62], and derives five more by extension and
puncturing.  Here the printed exponent lists are turned into generator
matrices: this module builds inputs only and holds none of the
minimum-distance arithmetic (no rank, no information sets, no
enumeration).

Conventions.  Coordinate i of a block holds the coefficient of x^i; block 1
is coordinates 0..m-1, block 2 is m..2m-1.  The generator rows are
x^i f_1 -> (x^i f_1, x^i f_1 p) for i < m - deg f_1, then
x^i f_2 -> (0, x^i f_2) for i < m - deg f_2.  p is reduced modulo
x^m - 1 (x^m = 1) where its printed degree reaches m.  Extension appends the
overall parity coordinate (the sum of a row's bits); puncturing deletes
coordinates, numbered from 1 as in the section's table (coordinate n is the
last one).  Reversing the coefficient order, or shifting both blocks
together, maps the code to an equivalent one (the simultaneous cyclic shift
maps the code to itself), so neither choice changes a distance; puncturing
at the last coordinate, or the last two, is the same up to equivalence under
either order.

Layout of the returned matrices: k rows of ceil(n/64) uint64 words, column c
at bit c % 64 of word c // 64, padding bits zero (the library's layout).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

M = 117

# f_1 (degree 67), common to both base codes
F1 = (67, 59, 54, 51, 49, 42, 39, 36, 35, 34, 33, 31, 30, 29, 27, 26, 25, 24,
      22, 21, 19, 17, 16, 15, 14, 13, 11, 6, 5, 3, 2, 0)

# the unit p of the [234,51] code (printed degree 117: x^117 = 1)
P_234_51 = (117, 116, 115, 111, 110, 109, 103, 102, 98, 95, 94, 92, 88, 85, 83,
            81, 74, 72, 70, 68, 66, 65, 64, 62, 61, 58, 56, 55, 54, 51, 49, 45,
            43, 39, 38, 37, 36, 35, 34, 28, 27, 23, 22, 20, 19, 16, 14, 9, 7,
            6, 5, 4, 3, 2, 0)

# the unit p of the [234,52] code (printed degree 217)
P_234_52 = (217, 214, 213, 211, 210, 209, 207, 205, 203, 202, 200, 198, 195,
            194, 193, 192, 190, 189, 186, 185, 183, 182, 180, 176, 175, 173,
            172, 171, 169, 167, 165, 164, 161, 160, 159, 155, 154, 151, 150,
            148, 147, 144, 143, 142, 141, 140, 137, 135, 132, 130, 129, 128,
            127, 125, 124, 122, 121, 119, 118, 116, 112, 107, 105, 103, 102,
            99, 97, 90, 89, 88, 87, 82, 76, 74, 71, 69, 68, 66, 64, 60, 53, 51,
            50, 47, 45, 43, 40, 39, 37, 36, 35, 34, 33, 31, 30, 29, 28, 26, 24,
            21, 20, 18, 17, 15, 14, 12, 8, 5, 4, 3, 0)


def poly(exponents) -> np.ndarray:
    """Coefficient vector (index = exponent) of a sum of distinct monomials."""
    a = np.zeros(max(exponents) + 1, dtype=np.uint8)
    for e in exponents:
        a[e] ^= 1
    return a


def pmul(a, b) -> np.ndarray:
    """Product in F_2[x] (no reduction)."""
    out = np.zeros(len(a) + len(b) - 1, dtype=np.uint8)
    for i in np.nonzero(a)[0]:
        out[i:i + len(b)] ^= b
    return out


def pdivmod(a, b):
    """Quotient and remainder in F_2[x]; b must have a nonzero leading term."""
    a = np.array(a, dtype=np.uint8)
    db = int(np.nonzero(b)[0].max())
    b = np.asarray(b[:db + 1], dtype=np.uint8)
    q = np.zeros(max(len(a) - db, 1), dtype=np.uint8)
    for i in range(len(a) - 1, db - 1, -1):
        if a[i]:
            q[i - db] = 1
            a[i - db:i + 1] ^= b
    return q, a[:db] if db else np.zeros(0, dtype=np.uint8)


def reduce_cyclic(a, m: int = M) -> np.ndarray:
    """a modulo x^m - 1: the coefficient of x^e is added to x^(e mod m)."""
    out = np.zeros(m, dtype=np.uint8)
    for e in np.nonzero(a)[0]:
        out[e % m] ^= 1
    return out


def x_m_minus_1_over(divisor_exponents, m: int = M) -> np.ndarray:
    """(x^m - 1) / d(x), checked to divide exactly (over F_2, -1 = +1)."""
    q, r = pdivmod(poly((m, 0)), poly(divisor_exponents))
    if r.any():
        raise ValueError("divisor does not divide x^m - 1")
    return q[:int(np.nonzero(q)[0].max()) + 1]


def cyclic_rows(g, m: int = M) -> np.ndarray:
    """Rows x^i g(x), i < m - deg g, as length-m coefficient vectors."""
    deg = int(np.nonzero(g)[0].max())
    rows = np.zeros((m - deg, m), dtype=np.uint8)
    for i in range(m - deg):
        rows[i, i:i + deg + 1] = g[:deg + 1]
    return rows


def matrix_product_bits(f1, f2, p, m: int = M) -> np.ndarray:
    """0/1 generator matrix of [C_1 C_2] . [[1, p], [0, 1]], C_i = (f_i)."""
    p = reduce_cyclic(p, m)
    top = cyclic_rows(f1, m)
    bottom = cyclic_rows(f2, m)
    rows = []
    for c in top:
        rows.append(np.concatenate([c, reduce_cyclic(pmul(c, p), m)]))
    for c in bottom:
        rows.append(np.concatenate([np.zeros(m, dtype=np.uint8), c]))
    return np.array(rows, dtype=np.uint8)


def extend(bits) -> np.ndarray:
    """Append the overall parity coordinate."""
    bits = np.asarray(bits, dtype=np.uint8)
    return np.concatenate([bits, (bits.sum(axis=1) % 2).astype(np.uint8)[:, None]], axis=1)


def puncture(bits, coords_from_1) -> np.ndarray:
    """Delete coordinates, numbered from 1."""
    bits = np.asarray(bits, dtype=np.uint8)
    drop = set(coords_from_1)
    keep = [c for c in range(bits.shape[1]) if c + 1 not in drop]
    return bits[:, keep]


def pack(bits) -> np.ndarray:
    """(k, n) 0/1 array -> (k, ceil(n/64)) uint64, column c at bit c % 64 of word c // 64."""
    bits = np.asarray(bits, dtype=np.uint8)
    k, n = bits.shape
    W = (n + 63) // 64
    padded = np.zeros((k, 64 * W), dtype=np.uint64)
    padded[:, :n] = bits
    weights = np.uint64(1) << np.arange(64, dtype=np.uint64)
    return (padded.reshape(k, W, 64) * weights).sum(axis=2, dtype=np.uint64)


def base_code_bits(k: int) -> np.ndarray:
    """[234,51] (f_2 = (x^117-1)/(x+1)) or [234,52] (f_2 = (x^117-1)/(x^2+x+1))."""
    f1 = poly(F1)
    if k == 51:
        return matrix_product_bits(f1, x_m_minus_1_over((1, 0)), poly(P_234_51))
    if k == 52:
        return matrix_product_bits(f1, x_m_minus_1_over((2, 1, 0)), poly(P_234_52))
    raise ValueError("the section prints base codes of dimension 51 and 52 only")


@dataclass(frozen=True)
class NewCode:
    """One code of the section: parameters it claims, the code of the
    previously best known parameters it improves on, and how it is made."""
    name: str
    n: int
    k: int
    d: int              # the distance the section claims
    d_before: int       # the best previously known distance for [n, k]
    recipe: str         # "base", "extend:<name>", "puncture:<name>:<coords>"

    def bits(self) -> np.ndarray:
        kind, *rest = self.recipe.split(":")
        if kind == "base":
            b = base_code_bits(self.k)
        elif kind == "extend":
            b = extend(NEW_CODES[rest[0]].bits())
        elif kind == "puncture":
            b = puncture(NEW_CODES[rest[0]].bits(), [int(c) for c in rest[1].split(",")])
        else:
            raise ValueError(self.recipe)
        if b.shape != (self.k, self.n):
            raise AssertionError(f"{self.name}: built {b.shape}, expected {(self.k, self.n)}")
        return b

    def matrix(self) -> np.ndarray:
        return pack(self.bits())


# Section 6's codes.  The five derived ones are those whose timings the
# section's tables report; the table of derived codes prints the length of
# the twice-punctured code as 233, which deleting two coordinates of a
# length-234 code cannot give: it is [232,51,61] (the length its "from"
# column and the timing tables use).
NEW_CODES = {
    "mp234x51": NewCode("mp234x51", 234, 51, 63, 62, "base"),
    "mp234x52": NewCode("mp234x52", 234, 52, 62, 61, "base"),
    "mp235x51": NewCode("mp235x51", 235, 51, 64, 62, "extend:mp234x51"),
    "mp236x51": NewCode("mp236x51", 236, 51, 64, 63, "extend:mp235x51"),
    "mp233x51": NewCode("mp233x51", 233, 51, 62, 61, "puncture:mp234x51:234"),
    "mp232x51": NewCode("mp232x51", 232, 51, 61, 60, "puncture:mp234x51:234,233"),
    "mp233x52": NewCode("mp233x52", 233, 52, 61, 60, "puncture:mp234x52:234"),
}
