// mindist_kernels.hip -- gfx950 kernels of the minimum-distance enumeration.
//
// enum_pair_kernel computes, for one pair (Gamma_j, w) of Algorithm 1, the
// least weight of c*Gamma_j over all c with wt(c) = w (the inner minimum of
// Algorithm 1), with the left/right split described in mindist_internal.h.
// The hot loop per codeword is: D x v_xor_b32 (lane row sum ^ scalar right
// sum), D x v_bcnt_u32_b32 (accumulating popcount), one v_min_u32.  Rows and
// tables are a few KB to a few MB; nothing per codeword touches HBM.
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
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += (uint64_t)__shfl_xor((long long)v, o);
    return uni64(v);
}

// Colex unranking: the a-subset {x_1 < ... < x_a} of [0, hi) with
// sum_t C(x_t, t) = rho.  Adds the rows of the subset into acc and returns
// the largest element.
template <int D>
__device__ __forceinline__ int unrank_add(const uint64_t *bt, const uint32_t *rows, int dp,
                                          uint64_t rho, int a, int hi, uint32_t (&acc)[D],
                                          bool reflect, int k) {
    int top = -1;
    for (int t = a; t >= 1; --t) {
        int lo = t - 1, h = hi - 1;
        while (lo < h) {
            int mid = (lo + h + 1) >> 1;
            if (binom(bt, mid, t) <= rho) lo = mid; else h = mid - 1;
        }
        rho -= binom(bt, lo, t);
        hi = lo;
        if (top < 0) top = lo;
        const int r = reflect ? (k - 1 - lo) : lo;
#pragma unroll
        for (int d = 0; d < D; ++d) acc[d] ^= rows[(size_t)r * dp + d];
    }
    return top;
}

// ---------------------------------------------------------------------------
// Run codewords [i0, i1) of the right table against the B lane items.
//   PRED: mask item t once i >= nr[t] (its right range ended)
//   SUM : accumulate weights (verify mode)
//   vm  : per item 0xFFFFFFFF if the item counts, 0 for a clamped duplicate
template <int D, int B, bool PRED, bool SUM>
__device__ __forceinline__ void run_range(const uint32_t *tab, uint32_t i0, uint32_t i1,
                                          const uint32_t (&L)[B][D], const uint32_t (&nr)[B],
                                          const uint32_t (&vm)[B], uint32_t (&m)[B],
                                          uint32_t &ws) {
    constexpr int DP = dp_of(D);
    cu32 *ct = (cu32 *)tab;
#pragma unroll 4
    for (uint32_t i = i0; i < i1; ++i) {
        uint32_t s[D];
#pragma unroll
        for (int d = 0; d < D; ++d) s[d] = ct[(size_t)i * DP + d];
#pragma unroll
        for (int t = 0; t < B; ++t) {
            uint32_t w = 0;
#pragma unroll
            for (int d = 0; d < D; ++d) w = __builtin_popcount(L[t][d] ^ s[d]) + w;
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
}

template <int D, int B, bool VERIFY>
__global__ __launch_bounds__(256) void enum_pair_kernel(PairArgs p) {
    constexpr int DP = dp_of(D);
    const int lane = threadIdx.x & 63;
    const uint64_t TB = 64ull * B;
    PairStat *ps = state_pairs(p.st) + p.pair;
    Slot *slots = state_slots(p.st);
    int gi = 0;
    for (;;) {
        uint64_t c = 0;
        if (lane == 0) c = atomicAdd((unsigned long long *)&ps->next_chunk, 1ull);
        c = uni64((uint64_t)__shfl((long long)c, 0));
        if (c >= p.total_chunks) break;
        if (p.midpair_exit &&
            __hip_atomic_load(&p.st->exit_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            break;
        if (p.cancel_after) {
            uint64_t cl = 0;
            if (lane == 0) cl = atomicAdd((unsigned long long *)&p.st->claimed, 1ull);
            cl = uni64((uint64_t)__shfl((long long)cl, 0));
            if (cl >= p.cancel_after) {
                if (lane == 0) atomicExch(&p.st->cancelled, 1u);
                break;
            }
        }
        // chunk -> (left tile, right tile); chunk ids of a wave only grow
        while (gi + 1 < p.ngroups && p.groups[gi + 1].chunk_base <= c) ++gi;
        const GroupEntry g = p.groups[gi];
        const uint64_t off = c - g.chunk_base;
        const uint64_t lt = g.lt_begin + off / g.n_rt;
        const uint32_t rt = (uint32_t)(off % g.n_rt);
        const uint32_t i_begin = rt * p.T;
        const uint32_t i_end = min(i_begin + p.T, g.nr_first);

        // lane items: left subsets rho = lt*64B + t*64 + lane (clamped to the
        // last valid item, which then counts once)
        uint32_t L[B][D];
        uint32_t nr[B];
        uint64_t rho_c[B];
        bool valid[B];
        uint32_t nr_lane_min = kInf;
#pragma unroll
        for (int t = 0; t < B; ++t) {
            const uint64_t rho = lt * TB + (uint64_t)t * 64 + lane;
            valid[t] = rho < p.n_items;
            rho_c[t] = valid[t] ? rho : p.n_items - 1;
#pragma unroll
            for (int d = 0; d < D; ++d) L[t][d] = 0;
            const int e = unrank_add<D>(p.binom, p.rows, DP, rho_c[t], p.a, p.k, L[t], false, p.k);
            nr[t] = (uint32_t)binom(p.binom, p.k - 1 - e, p.b);
            nr_lane_min = min(nr_lane_min, nr[t]);
        }
        const uint32_t nr_min = wave_min_u32(nr_lane_min);
        const uint32_t fast_end = min(i_end, max(i_begin, nr_min));

        uint32_t m[B], vm[B];
#pragma unroll
        for (int t = 0; t < B; ++t) {
            m[t] = kInf;
            vm[t] = valid[t] ? kInf : 0u;
        }
        uint32_t ws = 0;
        run_range<D, B, false, VERIFY>(p.table, i_begin, fast_end, L, nr, vm, m, ws);
        run_range<D, B, true, VERIFY>(p.table, fast_end, i_end, L, nr, vm, m, ws);

        uint64_t cnt = 0;
        uint32_t lmin = kInf;
#pragma unroll
        for (int t = 0; t < B; ++t) {
            lmin = min(lmin, m[t]);
            if (valid[t]) {
                const uint32_t hi = min(i_end, nr[t]);
                cnt += hi > i_begin ? (uint64_t)(hi - i_begin) : 0ull;
            }
        }
        const uint32_t wmin = wave_min_u32(lmin);
        const uint64_t wcnt = wave_sum_u64(cnt);
        uint64_t wws = 0;
        if (VERIFY) wws = wave_sum_u64((uint64_t)ws);
        if (lane == 0) {
            atomicAdd((unsigned long long *)&ps->executed, (unsigned long long)wcnt);
            if (VERIFY)
                atomicAdd((unsigned long long *)&ps->wsum,
                          (unsigned long long)(wws + (uint64_t)p.offset * wcnt));
            if (wmin != kInf) atomicMin(&ps->pair_min, wmin + p.offset);
        }
        if (wmin == kInf) continue;
        const uint32_t val = wmin + p.offset;
        const uint32_t cur =
            __hip_atomic_load(&p.st->U_found, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (val >= cur) continue;
        uint32_t old = 0;
        if (lane == 0) old = atomicMin(&p.st->U_found, val);
        old = uni32((uint32_t)__shfl((int)old, 0));
        if (old > val) {
            // this wave moved U_found to val: it alone writes slot[val].
            // Find the first (item, i) of the chunk that has weight wmin.
            uint32_t hit_i = kInf;
            int hit_t = -1;
            cu32 *ct = (cu32 *)p.table;
            for (uint32_t i = i_begin; i < i_end && hit_t < 0; ++i) {
                uint32_t s[D];
#pragma unroll
                for (int d = 0; d < D; ++d) s[d] = ct[(size_t)i * DP + d];
#pragma unroll
                for (int t = 0; t < B; ++t) {
                    uint32_t w = 0;
#pragma unroll
                    for (int d = 0; d < D; ++d) w = __builtin_popcount(L[t][d] ^ s[d]) + w;
                    if (hit_t < 0 && i < nr[t] && w == wmin) { hit_t = t; hit_i = i; }
                }
            }
            const unsigned long long ball = __ballot(hit_t >= 0);
            const int first = ball ? __builtin_ctzll(ball) : -1;
            if (lane == first) {
                uint64_t rho = 0;
#pragma unroll
                for (int t = 0; t < B; ++t) if (t == hit_t) rho = rho_c[t];
                slots[val].pair = p.pair;
                slots[val].i = hit_i;
                slots[val].rho = rho;
            }
        }
        if (p.midpair_exit && val <= p.L_prev && lane == 0)
            __hip_atomic_store(&p.st->exit_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Right table: entry i = sum of the rows {k-1-z : z in colex_unrank_b(i)}.
template <int D>
__global__ __launch_bounds__(256) void build_table_kernel(TableArgs ta) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ta.entries) return;
    uint32_t acc[D];
#pragma unroll
    for (int d = 0; d < D; ++d) acc[d] = 0;
    unrank_add<D>(ta.binom, ta.rows, ta.dp, i, ta.b, ta.k, acc, true, ta.k);
#pragma unroll
    for (int d = 0; d < D; ++d) ta.table[i * ta.dp + d] = acc[d];
    for (int d = D; d < ta.dp; ++d) ta.table[i * ta.dp + d] = 0;
}

__global__ void init_state_kernel(DevState *st, int max_pairs) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if (tid == 0) {
        st->U_found = kInf;
        st->exit_flag = 0;
        st->cancelled = 0;
        st->claimed = 0;
    }
    PairStat *ps = state_pairs(st);
    for (int p = tid; p < max_pairs; p += gridDim.x * blockDim.x) {
        ps[p].pair_min = kInf;
        ps[p].executed = 0;
        ps[p].wsum = 0;
        ps[p].next_chunk = 0;
    }
}

// ---------------------------------------------------------------------------
constexpr int kB = 2;   // lane items per chunk

int max_dwords() { return 16; }

static int check(hipError_t e) { return e == hipSuccess ? 0 : -1; }

int launch_init_state(DevState *st, int max_pairs, void *stream) {
    hipLaunchKernelGGL(init_state_kernel, dim3(64), dim3(256), 0, (hipStream_t)stream, st,
                       max_pairs);
    return check(hipGetLastError());
}

template <int D>
static void table_launch(const TableArgs &ta, hipStream_t s) {
    const uint64_t blocks = (ta.entries + 255) / 256;
    hipLaunchKernelGGL(build_table_kernel<D>, dim3((unsigned)blocks), dim3(256), 0, s, ta);
}

int launch_build_table(const TableArgs &ta, int D, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    switch (D) {
#define MD_CASE(X) case X: table_launch<X>(ta, s); break;
        MD_CASE(1) MD_CASE(2) MD_CASE(3) MD_CASE(4) MD_CASE(5) MD_CASE(6) MD_CASE(7) MD_CASE(8)
        MD_CASE(9) MD_CASE(10) MD_CASE(11) MD_CASE(12) MD_CASE(13) MD_CASE(14) MD_CASE(15)
        MD_CASE(16)
#undef MD_CASE
        default: return -2;
    }
    return check(hipGetLastError());
}

template <int D>
static void enum_launch(const PairArgs &pa, int verify, int blocks, hipStream_t s) {
    if (verify)
        hipLaunchKernelGGL((enum_pair_kernel<D, kB, true>), dim3(blocks), dim3(256), 0, s, pa);
    else
        hipLaunchKernelGGL((enum_pair_kernel<D, kB, false>), dim3(blocks), dim3(256), 0, s, pa);
}

int launch_enum_pair(const PairArgs &pa, int D, int verify, int blocks, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    switch (D) {
#define MD_CASE(X) case X: enum_launch<X>(pa, verify, blocks, s); break;
        MD_CASE(1) MD_CASE(2) MD_CASE(3) MD_CASE(4) MD_CASE(5) MD_CASE(6) MD_CASE(7) MD_CASE(8)
        MD_CASE(9) MD_CASE(10) MD_CASE(11) MD_CASE(12) MD_CASE(13) MD_CASE(14) MD_CASE(15)
        MD_CASE(16)
#undef MD_CASE
        default: return -2;
    }
    return check(hipGetLastError());
}

}  // namespace md
