"""Seeded synthetic inputs: random binary generator matrices.

This module only draws random bits; it holds none of the minimum-distance
arithmetic (no rank, no elimination, no enumeration).  Both the CPU oracle
(tests) and the HIP path read matrices produced here, and nothing else is
shared between them.

Random source: PCG32 (O'Neill 2014, "PCG: A family of simple fast
space-efficient statistically good algorithms for random number
generation"), the XSH-RR 64/32 member with the seeding procedure of the
published ``pcg32_srandom_r``: state = 0, inc = 2*stream+1, one step,
state += seed, one step.  Bounded integers use the published
``pcg32_boundedrand_r`` rejection rule.

Layout of a generated matrix: k rows of W = ceil(n/64) uint64 words, column
c at bit c % 64 of word c // 64 (LSB first), bits >= n are zero.  Each word
is two consecutive 32-bit draws, low half first; rows are drawn in order,
row-major.  ``attempt`` t skips the draws of attempts 0..t-1 of the same
stream, so a resampled matrix is simply a later attempt.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_MULT = np.uint64(6364136223846793005)
_M64 = (1 << 64) - 1


class PCG32:
    """PCG32 XSH-RR generator with vectorised draws (LCG jump-ahead)."""

    _jump_n = 0
    _jump_a: np.ndarray | None = None   # a^t mod 2^64
    _jump_s: np.ndarray | None = None   # sum_{i<t} a^i mod 2^64

    def __init__(self, seed: int, stream: int = 0):
        self.inc = ((stream << 1) | 1) & _M64
        self.state = 0
        self._step()
        self.state = (self.state + seed) & _M64
        self._step()

    def _step(self) -> int:
        old = self.state
        self.state = (old * 6364136223846793005 + self.inc) & _M64
        return old

    @staticmethod
    def _out(old: int) -> int:
        xs = (((old >> 18) ^ old) >> 27) & 0xFFFFFFFF
        rot = old >> 59
        return ((xs >> rot) | (xs << ((-rot) & 31))) & 0xFFFFFFFF

    def next_u32(self) -> int:
        return self._out(self._step())

    def bounded(self, bound: int) -> int:
        """Uniform integer in [0, bound) by rejection (pcg32_boundedrand_r)."""
        threshold = ((1 << 32) - bound) % bound
        while True:
            r = self.next_u32()
            if r >= threshold:
                return r % bound

    def uniform_int(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        return lo + self.bounded(hi - lo + 1)

    @classmethod
    def _ensure_jump(cls, n: int) -> None:
        if n <= cls._jump_n:
            return
        n = max(n, 2 * cls._jump_n, 4096)
        a = np.empty(n + 1, dtype=np.uint64)
        s = np.empty(n + 1, dtype=np.uint64)
        a[0], s[0] = 1, 0
        with np.errstate(over="ignore"):
            for t in range(1, n + 1):
                a[t] = a[t - 1] * _MULT
                s[t] = s[t - 1] * _MULT + np.uint64(1)
        cls._jump_a, cls._jump_s, cls._jump_n = a, s, n

    def draws(self, count: int) -> np.ndarray:
        """The next `count` 32-bit outputs as a uint32 array."""
        if count == 0:
            return np.zeros(0, dtype=np.uint32)
        self._ensure_jump(count)
        a = self._jump_a[:count + 1]
        s = self._jump_s[:count + 1]
        with np.errstate(over="ignore"):
            st = a * np.uint64(self.state) + np.uint64(self.inc) * s
        old = st[:count]
        xs = (((old >> np.uint64(18)) ^ old) >> np.uint64(27)) & np.uint64(0xFFFFFFFF)
        rot = old >> np.uint64(59)
        left = (np.uint64(32) - rot) & np.uint64(31)
        out = ((xs >> rot) | (xs << left)) & np.uint64(0xFFFFFFFF)
        self.state = int(st[count])
        return out.astype(np.uint32)


def words_per_row(n: int) -> int:
    return (n + 63) // 64


def draw_matrix(rng: PCG32, n: int, k: int) -> np.ndarray:
    """One k x n Bernoulli(1/2) matrix, packed (k, W) uint64, padding zero."""
    W = words_per_row(n)
    d = rng.draws(2 * k * W).astype(np.uint64)
    words = (d[0::2] | (d[1::2] << np.uint64(32))).reshape(k, W)
    rem = n - 64 * (W - 1)
    if rem < 64:
        words[:, W - 1] &= np.uint64((1 << rem) - 1)
    return words


def random_generator(n: int, k: int, seed: int, stream: int = 0,
                     attempt: int = 0) -> np.ndarray:
    """Attempt `attempt` of a seeded k x n random generator matrix."""
    if not (1 <= k < n <= 512):
        raise ValueError("need 1 <= k < n <= 512")
    rng = PCG32(seed, stream)
    if attempt:
        rng.draws(2 * k * words_per_row(n) * attempt)
    return draw_matrix(rng, n, k)


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    k: int
    seed: int
    stream: int
    attempt: int   # first attempt that meets the acceptance rule (see doc)

    def matrix(self) -> np.ndarray:
        return random_generator(self.n, self.k, self.seed, self.stream,
                                self.attempt)


# Single-code workloads.  Acceptance rules (checked against the CPU oracle
# by tests/golden/make_golden.py, which wrote these attempt numbers):
#   rand48x24   : rank 24 and the greedy partition gives 2 full information
#                 sets (no partial set),
#   rand150x75  : rank 75 and 2 full information sets,
#   rand255x40  : rank 40, exactly 6 full information sets and a partial
#                 set of rank >= 1.
WORKLOADS = {
    "rand48x24": Workload("rand48x24", 48, 24, 1, 0, 0),
    "rand150x75": Workload("rand150x75", 150, 75, 2, 0, 6),
    "rand255x40": Workload("rand255x40", 255, 40, 3, 0, 0),
}


# Sizes of the random codes the paper times (Tables 1, 2 and 4), with the
# distance it reports.  Their matrices are not published; paper_random_code
# draws a seeded stand-in of the same [n, k] (seed 6, stream 1000 n + k).
PAPER_RANDOM_SIZES = ((150, 50, 28), (130, 67, 15), (115, 63, 11), (102, 62, 12), (150, 77, 17))


def paper_random_code(n: int, k: int, attempt: int = 0) -> np.ndarray:
    """Attempt `attempt` of the seeded stand-in for the paper's random [n, k]."""
    return random_generator(n, k, 6, 1000 * n + k, attempt)


def batch_code(index: int, seed: int = 4, n_lo: int = 64, n_hi: int = 160):
    """Code `index` of the batch stream: n ~ U{n_lo..n_hi},
    k ~ U{ceil(n/4)..floor(n/2)}, then the k x n matrix (stream = index)."""
    rng = PCG32(seed, index)
    n = rng.uniform_int(n_lo, n_hi)
    k = rng.uniform_int(math.ceil(n / 4), n // 2)
    return n, k, draw_matrix(rng, n, k)


def batch_codes(count: int, seed: int = 4, n_lo: int = 64, n_hi: int = 160):
    return [batch_code(i, seed, n_lo, n_hi) for i in range(count)]


def serving_request(index: int, seed: int = 5, n_lo: int = 48, n_hi: int = 200):
    """Request `index` of the serving stream: n ~ U{n_lo..n_hi},
    k ~ U{ceil(n/5)..floor(n/2)}, then the k x n matrix (stream = index)."""
    rng = PCG32(seed, index)
    n = rng.uniform_int(n_lo, n_hi)
    k = rng.uniform_int(math.ceil(n / 5), n // 2)
    return n, k, draw_matrix(rng, n, k)


def poisson_arrivals(count: int, rate: float, seed: int = 5,
                     stream: int = 1 << 40) -> np.ndarray:
    """Arrival times (s) of a Poisson process of `rate` per second: i.i.d.
    exponential gaps by inversion of 24-bit uniforms, on a stream of its own."""
    rng = PCG32(seed, stream)
    u = (rng.draws(count).astype(np.float64) // 256 + 0.5) / float(1 << 24)
    gaps = -np.log(u) / rate
    return np.cumsum(gaps)
