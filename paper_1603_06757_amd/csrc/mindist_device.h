// mindist_device.h -- device helpers shared by the enumeration kernels: the
// per-chunk work of one pair (left subsets per lane, right sums by scalar
// loads, one XOR + popcount per carried word) and the witness search.
//
// Per codeword the vector-ALU loop issues D x v_xor_b32 (lane row sum ^
// scalar right sum), D x v_bcnt_u32_b32 (accumulating popcount) and half a
// v_min3_u32.  Up to 4 words the part of a chunk every lane subset covers
// runs instead as int8 products on the matrix cores (run_range_mfma).
#pragma once
#include <hip/hip_runtime.h>

#include "mindist_internal.h"

namespace md {

typedef const __attribute__((address_space(4))) uint32_t cu32;

__host__ __device__ constexpr int dp_of(int D) {
    return D <= 1 ? 1 : D <= 2 ? 2 : D <= 4 ? 4 : D <= 8 ? 8 : 16;
}

__device__ __forceinline__ uint64_t binom(const uint64_t *bt, int x, int t) {
    return (x < 0 || t < 0 || t > x) ? 0ull : bt[x * kBinomT + t];
}

__device__ __forceinline__ uint32_t uni32(uint32_t v) {
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
    return uni32(v);
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o));
    return uni32(v);
}
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t u = (uint64_t)__shfl_xor((long long)v, o);
        v = u < v ? u : v;
    }
    return uni64(v);
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t u = (uint64_t)__shfl_xor((long long)v, o);
        v = u > v ? u : v;
    }
    return uni64(v);
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += (uint64_t)__shfl_xor((long long)v, o);
    return uni64(v);
}

// Colex unranking: the a-subset {x_1 < ... < x_a} of [0, hi) with
// sum_t C(x_t, t) = rho.  Adds the rows of the subset into acc and returns
// the largest element.  bt holds C(x, t) at bt[x * bs + t] for t <= a and
// x < hi (zero for t > x): the full table (bs = kBinomT) or a slice of it.
template <int D>
__device__ __forceinline__ int unrank_add(const uint64_t *bt, int bs, const uint32_t *rows, int dp,
                                          uint64_t rho, int a, int hi, uint32_t (&acc)[D],
                                          bool reflect, int k) {
    int top = -1;
    for (int t = a; t >= 1; --t) {
        int lo = t - 1, h = hi - 1;
        while (lo < h) {
            int mid = (lo + h + 1) >> 1;
            if (bt[mid * bs + t] <= rho) lo = mid; else h = mid - 1;
        }
        rho -= bt[lo * bs + t];
        hi = lo;
        if (top < 0) top = lo;
        const int r = reflect ? (k - 1 - lo) : lo;
#pragma unroll
        for (int d = 0; d < D; ++d) acc[d] ^= rows[(size_t)r * dp + d];
    }
    return top;
}

// v_bcnt_u32_b32 with its accumulator operand: popcount(x) + acc in one
// instruction (the compiler would otherwise sum separate popcounts with
// v_add3, one more instruction per codeword).
__device__ __forceinline__ uint32_t bcnt_acc(uint32_t x, uint32_t acc) {
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

template <int D>
__device__ __forceinline__ uint32_t weight_of(const uint32_t (&L)[D], const uint32_t (&s)[D]) {
    uint32_t w = __builtin_popcount(L[0] ^ s[0]);
#pragma unroll
    for (int d = 1; d < D; ++d) w = bcnt_acc(L[d] ^ s[d], w);
    return w;
}

// A right-table entry is dp_of(D) words; it is fetched whole (the padding
// word of D = 3 included) so one scalar load brings one entry.
template <int DP> struct Entry { uint32_t w[DP]; };
template <> struct Entry<4> {
    typedef uint32_t v4 __attribute__((ext_vector_type(4)));
    v4 v;
};
template <int D>
__device__ __forceinline__ void load_entry(cu32 *ct, uint32_t i, uint32_t (&s)[D]) {
    constexpr int DP = dp_of(D);
    if constexpr (DP == 4) {
        typedef const __attribute__((address_space(4))) Entry<4>::v4 cv4;
        const Entry<4>::v4 v = ((cv4 *)ct)[i];
        s[0] = v.x;
        if constexpr (D > 1) s[1] = v.y;
        if constexpr (D > 2) s[2] = v.z;
        if constexpr (D > 3) s[3] = v.w;
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) s[d] = ct[(size_t)i * DP + d];
    }
}

// right-table entries per pipelined block (two blocks live in SGPRs)
template <int D>
__host__ __device__ constexpr int block_of() { return dp_of(D) <= 4 ? 4 : dp_of(D) <= 8 ? 2 : 1; }

// One right-table entry against the B lane items.
//   PRED: mask item t once i >= nr[t] (its right range ended)
//   SUM : accumulate weights (verify mode); vm[t] = 0 drops a clamped
//         duplicate item from the sum
template <int D, int B, bool PRED, bool SUM>
__device__ __forceinline__ void step(const uint32_t (&s)[D], uint32_t i, const uint32_t (&L)[B][D],
                                     const uint32_t (&nr)[B], const uint32_t (&vm)[B],
                                     uint32_t (&m)[B], uint32_t &ws) {
#pragma unroll
    for (int t = 0; t < B; ++t) {
        uint32_t w = weight_of<D>(L[t], s);
        if (PRED) {
            const bool on = i < nr[t];
            if (SUM) ws += on ? (w & vm[t]) : 0u;
            w = on ? w : kInf;
        } else if (SUM) {
            ws += w & vm[t];
        }
        m[t] = min(m[t], w);
    }
}

// Run right-table entries [i0, i1) against the B lane items.  The uniform
// entries come in by scalar loads; the next block is requested before the
// current one is consumed so the load latency overlaps the VALU work.
template <int D, int B, bool PRED, bool SUM>
__device__ __forceinline__ void run_range(const uint32_t *tab, uint32_t i0, uint32_t i1,
                                          const uint32_t (&L)[B][D], const uint32_t (&nr)[B],
                                          const uint32_t (&vm)[B], uint32_t (&m)[B],
                                          uint32_t &ws) {
    constexpr int U = block_of<D>();
    cu32 *ct = (cu32 *)tab;
    uint32_t i = i0;
    if (i1 - i0 >= 2 * U) {
        uint32_t cur[U][D], nxt[U][D];
#pragma unroll
        for (int u = 0; u < U; ++u) load_entry<D>(ct, i + u, cur[u]);
        for (; i + 2 * U <= i1; i += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) load_entry<D>(ct, i + U + u, nxt[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) step<D, B, PRED, SUM>(cur[u], i + u, L, nr, vm, m, ws);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int d = 0; d < D; ++d) cur[u][d] = nxt[u][d];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) step<D, B, PRED, SUM>(cur[u], i + u, L, nr, vm, m, ws);
        i += U;
    }
    for (; i < i1; ++i) {
        uint32_t s[D];
        load_entry<D>(ct, i, s);
        step<D, B, PRED, SUM>(s, i, L, nr, vm, m, ws);
    }
}


// ---- the same minimum on the int8 matrix cores --------------------------
// For bit vectors l and r, wt(l ^ r) = wt(l) + sum_k r_k (1 - 2 l_k): the
// weight of every (left, right) combination is wt(l) plus an integer inner
// product, so a block of 32 right entries against 32 left subsets is one
// 32 x 32 product over k = 32 D bit positions -- D v_mfma_i32_32x32x32_i8,
// right bits as 0/1 bytes (rows), left bits as +1/-1 bytes (columns).
// Operand layout of that instruction: lane i + 32h holds k = 16h .. 16h+15
// of row (A) or column (B) i, one byte each, in both operands; result value
// r of lane l is row 8(r/4) + 4(l/32) + r%4 of column l%32.  Word d of a
// sum supplies k = 32d .. 32d+31, so a lane takes bits 16h .. 16h+15 of
// each word.  Exact: |inner product| <= 32 D.
typedef int mf_v4i __attribute__((ext_vector_type(4)));
typedef int mf_v16i __attribute__((ext_vector_type(16)));

// bits 4c .. 4c+3 of x as bytes 0/1 (bit 4c+p -> byte p)
__device__ __forceinline__ uint32_t bit_bytes4(uint32_t x, int c) {
    return __umul24((x >> (4 * c)) & 0xFu, 0x00204081u) & 0x01010101u;
}
// the 16 low bits of x as 16 bytes 0/1
__device__ __forceinline__ mf_v4i bits01(uint32_t x) {
    return mf_v4i{(int)bit_bytes4(x, 0), (int)bit_bytes4(x, 1), (int)bit_bytes4(x, 2), (int)bit_bytes4(x, 3)};
}
// the 16 low bits of x as 16 bytes +1 (clear) / -1 (set)
__device__ __forceinline__ mf_v4i bits_pm(uint32_t x) {
    mf_v4i v;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const uint32_t b = bit_bytes4(x, c);
        v[c] = (int)(((b << 8) - b) | 0x01010101u);   // 0xff per set bit, then 0x01 on every byte
    }
    return v;
}

// Right entries [i0, i0 + 32 nb) against the wave's 64 B left subsets (item t
// of lane u: L[t] of lane u), all of them in range: m[t] = min(m[t], least
// weight of item t).  Column tile q holds items t = q/2 of lanes
// 32(q%2) .. 32(q%2)+31.  CH: product chains in flight per wave, 1 or 2
// (tiles in pairs; faster where the registers allow it).
template <int D, int B, int CH>
__device__ __forceinline__ void run_range_mfma(const uint32_t *tab, uint32_t i0, uint32_t nb,
                                               const uint32_t (&L)[B][D], uint32_t (&m)[B]) {
    constexpr int DP = dp_of(D);
    constexpr int Q = 2 * B;
    const int lane = threadIdx.x & 63;
    const int h = lane >> 5;
    const uint32_t sh = 16u * (uint32_t)h;
    mf_v4i lb[Q][D];
#pragma unroll
    for (int t = 0; t < B; ++t)
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const uint32_t own = L[t][d];
            const uint32_t oth = (uint32_t)__shfl_xor((int)own, 32);
            lb[2 * t][d] = bits_pm((h ? oth : own) >> sh);       // column tile 2t: lanes 0..31's items
            lb[2 * t + 1][d] = bits_pm((h ? own : oth) >> sh);   // tile 2t+1: lanes 32..63's
        }
    int32_t rmin[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) rmin[q] = 0x7fffffff;
    // this lane's row of every block: entry i0 + 32b + lane%32.  The next
    // block's words are requested before the current block's products and
    // turned into bytes after them.  With CH = 2 tiles go in pairs, the two
    // products interleaved word by word (two independent chains); the minima
    // of one pair (or tile) are taken while the products of the next run.
    const uint32_t *rp = tab + (size_t)(i0 + (uint32_t)(lane & 31)) * DP;
    uint32_t nxt[D];
    mf_v4i ra[D];
#pragma unroll
    for (int d = 0; d < D; ++d) nxt[d] = rp[d];
#pragma unroll
    for (int d = 0; d < D; ++d) ra[d] = bits01(nxt[d] >> sh);
    for (uint32_t b = 0; b < nb; ++b) {
        const uint32_t *np = rp + (size_t)(b + 1 < nb ? b + 1 : b) * 32 * DP;
#pragma unroll
        for (int d = 0; d < D; ++d) nxt[d] = np[d];
        if constexpr (CH == 2) {
            mf_v16i p0 = {0}, p1 = {0};
#pragma unroll
            for (int d = 0; d < D; ++d) {
                p0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(ra[d], lb[0][d], p0, 0, 0, 0);
                p1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(ra[d], lb[1][d], p1, 0, 0, 0);
            }
#pragma unroll
            for (int q = 2; q <= Q; q += 2) {
                mf_v16i a0 = {0}, a1 = {0};
                if (q < Q) {
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        a0 = __builtin_amdgcn_mfma_i32_32x32x32_i8(ra[d], lb[q][d], a0, 0, 0, 0);
                        a1 = __builtin_amdgcn_mfma_i32_32x32x32_i8(ra[d], lb[q + 1][d], a1, 0, 0, 0);
                    }
                }
                int32_t v0 = rmin[q - 2], v1 = rmin[q - 1];
#pragma unroll
                for (int r = 0; r < 16; r += 2) {
                    v0 = min(min(v0, p0[r]), p0[r + 1]);
                    v1 = min(min(v1, p1[r]), p1[r + 1]);
                }
                rmin[q - 2] = v0;
                rmin[q - 1] = v1;
                p0 = a0;
                p1 = a1;
            }
        } else {
            mf_v16i prev = {0};
#pragma unroll
            for (int d = 0; d < D; ++d) prev = __builtin_amdgcn_mfma_i32_32x32x32_i8(ra[d], lb[0][d], prev, 0, 0, 0);
#pragma unroll
            for (int q = 1; q <= Q; ++q) {
                mf_v16i acc = {0};
                if (q < Q) {
#pragma unroll
                    for (int d = 0; d < D; ++d) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(ra[d], lb[q][d], acc, 0, 0, 0);
                }
                int32_t v = rmin[q - 1];
#pragma unroll
                for (int r = 0; r < 16; r += 2) v = min(min(v, prev[r]), prev[r + 1]);
                rmin[q - 1] = v;
                prev = acc;
            }
        }
#pragma unroll
        for (int d = 0; d < D; ++d) ra[d] = bits01(nxt[d] >> sh);
    }
    // column j of tile 2t+h is item t of lane 32h + j: this lane's own item;
    // its other 16 rows per block sit in lane ^ 32
#pragma unroll
    for (int t = 0; t < B; ++t) {
        const int32_t mine = h ? rmin[2 * t + 1] : rmin[2 * t];
        const int32_t theirs = __shfl_xor(h ? rmin[2 * t] : rmin[2 * t + 1], 32);
        uint32_t wl = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) wl += __builtin_popcount(L[t][d]);
        m[t] = min(m[t], (uint32_t)((int32_t)wl + min(mine, theirs)));
    }
}

// Where the left and right sums of one pair come from.  b is the size of the
// (outer) right subsets; b2 > 0 selects the three-level split with inner
// subsets of size b2 from table2.
struct ItemSrc {
    const uint32_t *rows;      // k x DP
    const uint32_t *table;     // right (outer) table
    const uint32_t *ltable;    // left table or nullptr (lanes unrank)
    const uint64_t *binom;     // binomials for the unranking: C(x, t) = binom[x * bs + t]
    const uint64_t *colA;      // C(x, a) = colA[x * sA]
    const uint64_t *colB;      // C(x, b) = colB[x * sB]
    int sA, sB;
    uint64_t n_items;          // C(k-b-b2, a)
    int k, a, b;
    int b2;
    const uint32_t *table2;    // inner table
    const uint32_t *cnt2;      // inner entries of each outer entry
    int bs;                    // row stride of binom (kBinomT for the full table)
};

// The part of the pair one chunk covers: left tile lt, right entries
// [i_begin, i_end) (i_end is clipped to the tile's first item's range when
// clip is set), e_first a lower bound on the largest element of the tile.
struct ChunkGeo {
    uint64_t lt;
    uint32_t i_begin, i_end;
    uint32_t e_first;
    bool clip;
};

// One chunk: B left subsets per lane (ranks lt*64B + t*64 + lane, clamped to
// the last valid one) against right entries [i_begin, i_end).  Returns the
// lane's least weight (without the identity offset), the number of
// combinations it evaluated and (VERIFY) their weight sum; L and nr stay
// valid for a witness search.  MF (D <= 4, not with VERIFY): 0, or the
// product chains per wave (1 or 2) with which the range every item covers
// runs on the matrix cores, in whole blocks of 32 entries.
template <int D, int B, bool VERIFY, int MF = 0>
__device__ __forceinline__ void run_chunk(const ItemSrc &s, ChunkGeo &g, uint32_t (&L)[B][D],
                                          uint32_t (&nr)[B], uint32_t &lmin, uint64_t &cnt,
                                          uint32_t &ws) {
    constexpr int DP = dp_of(D);
    const int lane = threadIdx.x & 63;
    const uint64_t tile0 = g.lt * (64ull * B) + lane;
    uint32_t nr_lane_min = kInf, nr_lane_max = 0;
#pragma unroll
    for (int t = 0; t < B; ++t) {
        const uint64_t rho = tile0 + (uint64_t)t * 64;
        const uint64_t rc = rho < s.n_items ? rho : s.n_items - 1;
#pragma unroll
        for (int d = 0; d < D; ++d) L[t][d] = 0;
        int e;
        if (s.ltable) {
            // saved left sum; its largest element e is the largest x with
            // C(x, a) <= rho (colex order sorts by largest element)
#pragma unroll
            for (int d = 0; d < D; ++d) L[t][d] = s.ltable[rc * DP + d];
            e = max((int)g.e_first, s.a - 1);
            int hi = s.k - 1 - s.b - s.b2;   // the largest e with a right partner
            while (e < hi) {
                const int mid = (e + hi + 1) >> 1;
                if (s.colA[(size_t)mid * s.sA] <= rc) e = mid; else hi = mid - 1;
            }
        } else {
            e = unrank_add<D>(s.binom, s.bs, s.rows, DP, rc, s.a, s.k, L[t], false, s.k);
        }
        nr[t] = (uint32_t)s.colB[(size_t)(s.k - 1 - e) * s.sB];
        nr_lane_min = min(nr_lane_min, nr[t]);
        nr_lane_max = max(nr_lane_max, nr[t]);
    }
    const uint32_t nr_min = wave_min_u32(nr_lane_min);
    if (g.clip) g.i_end = min(g.i_end, wave_max_u32(nr_lane_max));
    const uint32_t fast_end = min(g.i_end, max(g.i_begin, nr_min));

    uint32_t m[B], vm[B];
#pragma unroll
    for (int t = 0; t < B; ++t) {
        m[t] = kInf;
        vm[t] = (tile0 + (uint64_t)t * 64 < s.n_items) ? kInf : 0u;
    }
    ws = 0;
    uint32_t i_mid = g.i_begin;
    if constexpr (MF > 0) {
        // whole 32-entry blocks of the range every item covers on the matrix
        // cores, the rest on the VALU
        const uint32_t nb = (fast_end - g.i_begin) / 32;
        if (nb) run_range_mfma<D, B, MF>(s.table, g.i_begin, nb, L, m);
        i_mid = g.i_begin + 32 * nb;
    }
    run_range<D, B, false, VERIFY>(s.table, i_mid, fast_end, L, nr, vm, m, ws);
    run_range<D, B, true, VERIFY>(s.table, fast_end, g.i_end, L, nr, vm, m, ws);
    lmin = kInf;
    cnt = 0;
#pragma unroll
    for (int t = 0; t < B; ++t) {
        lmin = min(lmin, m[t]);
        if (tile0 + (uint64_t)t * 64 < s.n_items) {
            const uint32_t hi = min(g.i_end, nr[t]);
            cnt += hi > g.i_begin ? (uint64_t)(hi - g.i_begin) : 0ull;
        }
    }
}

// The first (item, entry) of the chunk whose weight is wmin: returns the lane
// that holds it (or -1), with its right index and left rank.
template <int D, int B>
__device__ __forceinline__ int find_witness(const ItemSrc &s, const ChunkGeo &g,
                                            const uint32_t (&L)[B][D], const uint32_t (&nr)[B],
                                            uint32_t wmin, uint32_t &hit_i, uint64_t &hit_rho) {
    const int lane = threadIdx.x & 63;
    hit_i = kInf;
    int hit_t = -1;
    cu32 *ct = (cu32 *)s.table;
#pragma unroll 1
    for (uint32_t i = g.i_begin; i < g.i_end && hit_t < 0; ++i) {
        uint32_t e[D];
        load_entry<D>(ct, i, e);
#pragma unroll
        for (int t = 0; t < B; ++t) {
            const uint32_t w = weight_of<D>(L[t], e);
            if (hit_t < 0 && i < nr[t] && w == wmin) { hit_t = t; hit_i = i; }
        }
    }
    const unsigned long long ball = __ballot(hit_t >= 0);
    const int first = ball ? __builtin_ctzll(ball) : -1;
    hit_rho = 0;
    if (lane == first) {
        const uint64_t tile0 = g.lt * (64ull * B) + lane;
#pragma unroll
        for (int t = 0; t < B; ++t)
            if (t == hit_t) {
                hit_rho = tile0 + (uint64_t)t * 64;
                if (hit_rho >= s.n_items) hit_rho = s.n_items - 1;
            }
    }
    return first;
}

// Inner loop of the three-level split: entries [0, n2) of the inner table
// against lane sums L2 (= left sum ^ outer entry); per item minimum and
// (SUM) weight sum.  Same pipelined scalar loads as run_range.
template <int D, int B, bool SUM>
__device__ __forceinline__ void run_inner(const uint32_t *tab, uint32_t n2, const uint32_t (&L2)[B][D],
                                          uint32_t (&mi)[B], uint32_t (&wsi)[B]) {
    constexpr int U = block_of<D>();
    cu32 *ct = (cu32 *)tab;
    uint32_t i = 0;
    if (n2 >= 2 * U) {
        uint32_t cur[U][D], nxt[U][D];
#pragma unroll
        for (int u = 0; u < U; ++u) load_entry<D>(ct, i + u, cur[u]);
        for (; i + 2 * U <= n2; i += U) {
#pragma unroll
            for (int u = 0; u < U; ++u) load_entry<D>(ct, i + U + u, nxt[u]);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int t = 0; t < B; ++t) {
                    const uint32_t w = weight_of<D>(L2[t], cur[u]);
                    if (SUM) wsi[t] += w;
                    mi[t] = min(mi[t], w);
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int d = 0; d < D; ++d) cur[u][d] = nxt[u][d];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int t = 0; t < B; ++t) {
                const uint32_t w = weight_of<D>(L2[t], cur[u]);
                if (SUM) wsi[t] += w;
                mi[t] = min(mi[t], w);
            }
        i += U;
    }
    for (; i < n2; ++i) {
        uint32_t e[D];
        load_entry<D>(ct, i, e);
#pragma unroll
        for (int t = 0; t < B; ++t) {
            const uint32_t w = weight_of<D>(L2[t], e);
            if (SUM) wsi[t] += w;
            mi[t] = min(mi[t], w);
        }
    }
}

// Lane items of a chunk: left sums L and outer range lengths nr; returns the
// wave-uniform min of nr and clips g.i_end (right-major order) to the max.
template <int D, int B>
__device__ __forceinline__ uint32_t setup_items(const ItemSrc &s, ChunkGeo &g, uint32_t (&L)[B][D],
                                                uint32_t (&nr)[B]) {
    constexpr int DP = dp_of(D);
    const int lane = threadIdx.x & 63;
    const uint64_t tile0 = g.lt * (64ull * B) + lane;
    uint32_t nr_lane_min = kInf, nr_lane_max = 0;
#pragma unroll
    for (int t = 0; t < B; ++t) {
        const uint64_t rho = tile0 + (uint64_t)t * 64;
        const uint64_t rc = rho < s.n_items ? rho : s.n_items - 1;
#pragma unroll
        for (int d = 0; d < D; ++d) L[t][d] = 0;
        int e;
        if (s.ltable) {
#pragma unroll
            for (int d = 0; d < D; ++d) L[t][d] = s.ltable[rc * DP + d];
            e = max((int)g.e_first, s.a - 1);
            int hi = s.k - 1 - s.b - s.b2;
            while (e < hi) {
                const int mid = (e + hi + 1) >> 1;
                if (s.colA[(size_t)mid * s.sA] <= rc) e = mid; else hi = mid - 1;
            }
        } else {
            e = unrank_add<D>(s.binom, s.bs, s.rows, DP, rc, s.a, s.k, L[t], false, s.k);
        }
        nr[t] = (uint32_t)s.colB[(size_t)(s.k - 1 - s.b2 - e) * s.sB];
        nr_lane_min = min(nr_lane_min, nr[t]);
        nr_lane_max = max(nr_lane_max, nr[t]);
    }
    if (g.clip) g.i_end = min(g.i_end, wave_max_u32(nr_lane_max));
    return wave_min_u32(nr_lane_min);
}

// One chunk of the three-level split: outer entries [i_begin, i_end) of
// table (b-subsets Y1), for each the inner entries [0, C(zmin, b2)) of
// table2.  Outputs as run_chunk.
template <int D, int B, bool VERIFY>
__device__ __forceinline__ void run_chunk3(const ItemSrc &s, ChunkGeo &g, uint32_t (&L)[B][D],
                                           uint32_t (&nr)[B], uint32_t &lmin, uint64_t &cnt,
                                           uint32_t &ws) {
    const int lane = threadIdx.x & 63;
    const uint64_t tile0 = g.lt * (64ull * B) + lane;
    const uint32_t nr_min = setup_items<D, B>(s, g, L, nr);
    const uint32_t fast_end = min(g.i_end, max(g.i_begin, nr_min));
    cu32 *ct = (cu32 *)s.table;
    cu32 *cn = (cu32 *)s.cnt2;
    uint32_t m[B];
    bool valid[B];
#pragma unroll
    for (int t = 0; t < B; ++t) {
        m[t] = kInf;
        valid[t] = tile0 + (uint64_t)t * 64 < s.n_items;
    }
    cnt = 0;
    ws = 0;
    for (uint32_t i1 = g.i_begin; i1 < g.i_end; ++i1) {
        uint32_t s1[D];
        load_entry<D>(ct, i1, s1);
        const uint32_t n2 = cn[i1];
        uint32_t L2[B][D], mi[B], wsi[B];
#pragma unroll
        for (int t = 0; t < B; ++t) {
            mi[t] = kInf;
            wsi[t] = 0;
#pragma unroll
            for (int d = 0; d < D; ++d) L2[t][d] = L[t][d] ^ s1[d];
        }
        run_inner<D, B, VERIFY>(s.table2, n2, L2, mi, wsi);
        const bool all_on = i1 < fast_end;
#pragma unroll
        for (int t = 0; t < B; ++t) {
            const bool on = all_on || i1 < nr[t];
            if (on) m[t] = min(m[t], mi[t]);
            if (on && valid[t]) {
                cnt += n2;
                if (VERIFY) ws += wsi[t];
            }
        }
    }
    lmin = kInf;
#pragma unroll
    for (int t = 0; t < B; ++t) lmin = min(lmin, m[t]);
}

// Three-level witness search: the first (item, i1, i2) of the chunk with
// weight wmin; returns the holding lane (or -1).
template <int D, int B>
__device__ __forceinline__ int find_witness3(const ItemSrc &s, const ChunkGeo &g,
                                             const uint32_t (&L)[B][D], const uint32_t (&nr)[B],
                                             uint32_t wmin, uint32_t &hit_i, uint32_t &hit_i2,
                                             uint64_t &hit_rho) {
    const int lane = threadIdx.x & 63;
    hit_i = hit_i2 = kInf;
    int hit_t = -1;
    cu32 *ct = (cu32 *)s.table;
    cu32 *c2 = (cu32 *)s.table2;
    // rare path (a new least weight): kept rolled so that it does not set
    // the kernel's register budget
#pragma unroll 1
    for (uint32_t i1 = g.i_begin; i1 < g.i_end && hit_t < 0; ++i1) {
        uint32_t s1[D];
        load_entry<D>(ct, i1, s1);
        const uint32_t n2 = s.cnt2[i1];
#pragma unroll 1
        for (uint32_t i2 = 0; i2 < n2 && hit_t < 0; ++i2) {
            uint32_t e[D];
            load_entry<D>(c2, i2, e);
#pragma unroll
            for (int d = 0; d < D; ++d) e[d] ^= s1[d];
#pragma unroll
            for (int t = 0; t < B; ++t) {
                const uint32_t w = weight_of<D>(L[t], e);
                if (hit_t < 0 && i1 < nr[t] && w == wmin) { hit_t = t; hit_i = i1; hit_i2 = i2; }
            }
        }
    }
    const unsigned long long ball = __ballot(hit_t >= 0);
    const int first = ball ? __builtin_ctzll(ball) : -1;
    hit_rho = 0;
    if (lane == first) {
        const uint64_t tile0 = g.lt * (64ull * B) + lane;
#pragma unroll
        for (int t = 0; t < B; ++t)
            if (t == hit_t) {
                hit_rho = tile0 + (uint64_t)t * 64;
                if (hit_rho >= s.n_items) hit_rho = s.n_items - 1;
            }
    }
    return first;
}

}  // namespace md
