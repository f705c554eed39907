// mindist_walk.hip -- the direct walk over one pair (Gamma_j, w), kept to
// measure the saved-sums enumeration against (the product path does not
// use it).
//
// Every lane takes its own run of consecutive ranks of the w-subsets in
// lexicographic order and starts independently: its first subset is
// unranked in the combinatorial number system (the number of subsets whose
// first element is x is C(k-1-x, w-1)).  It then walks the subsets in the
// order of the stack-based enumeration (Section 3.3, Algorithm 4): the
// partial sums S_i = rows c_0 + ... + c_i stay in registers, the last
// element runs over its remaining rows so that a codeword costs one row
// read from LDS, D XORs and D popcounts, and when it reaches row k-1 the
// rightmost element that can move advances, the elements after it follow
// it, and the partial sums from it on are rebuilt.  Lanes carry at
// different times, so the carry is divergent, and the inner run of the last
// element is short (about (k-w)/w rows), which is what the saved right sums
// of the product kernel avoid.
#include <hip/hip_runtime.h>

#include "mindist_device.h"
#include "mindist_walk.h"

namespace md {

template <int D>
__global__ __launch_bounds__(256) void walk_pair_kernel(WalkArgs a) {
    constexpr int DP = dp_of(D);
    __shared__ uint32_t s_rows[kWalkMaxK * DP];
    for (int i = threadIdx.x; i < a.k * DP; i += blockDim.x) s_rows[i] = a.rows[i];
    __syncthreads();

    const int k = a.k, w = a.w;
    const uint64_t lo = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * a.per_thread;
    const uint64_t hi = lo + a.per_thread < a.total ? lo + a.per_thread : a.total;
    uint32_t m = kInf;
    uint64_t done = 0;
    if (lo < hi) {
        // the subset of rank lo, c[0] < ... < c[w-1]
        int c[kWalkMaxW];
        uint64_t r = lo;
        int x = 0;
#pragma unroll
        for (int i = 0; i < kWalkMaxW; ++i) {
            c[i] = 0;
            if (i < w) {
                for (uint64_t b = binom(a.binom, k - 1 - x, w - 1 - i); b <= r && x < k - 1;
                     b = binom(a.binom, k - 1 - x, w - 1 - i)) {
                    r -= b;
                    ++x;
                }
                c[i] = x++;
            }
        }
        // partial sums of all elements but the last
        uint32_t S[kWalkMaxW][D];
        uint32_t pre[D];
#pragma unroll
        for (int d = 0; d < D; ++d) pre[d] = 0;
#pragma unroll
        for (int i = 0; i < kWalkMaxW; ++i) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                S[i][d] = (i < w - 1) ? ((i ? S[i - 1][d] : 0u) ^ s_rows[c[i] * DP + d]) : 0u;
                if (i == w - 2) pre[d] = S[i][d];
            }
        }
        int last = 0;
#pragma unroll
        for (int i = 0; i < kWalkMaxW; ++i)
            if (i == w - 1) last = c[i];

        uint64_t left = hi - lo;
        for (;;) {
            // the last element over rows last .. k-1 (or until the run ends)
            uint64_t run = (uint64_t)(k - last);
            if (run > left) run = left;
            for (uint32_t t = 0; t < (uint32_t)run; ++t) {
                const uint32_t *row = &s_rows[(last + t) * DP];
                uint32_t wt = a.offset;
#pragma unroll
                for (int d = 0; d < D; ++d) wt += __builtin_popcount(pre[d] ^ row[d]);
                m = min(m, wt);
            }
            left -= run;
            done += run;
            if (left == 0) break;
            // carry: the rightmost element before the last that can move
            int piv = -1;
#pragma unroll
            for (int i = 0; i < kWalkMaxW; ++i)
                if (i <= w - 2 && c[i] < k - (w - i)) piv = i;
            if (piv < 0) break;   // no later subset (cannot happen while ranks remain)
#pragma unroll
            for (int i = 0; i < kWalkMaxW; ++i) {
                if (i == piv) c[i] += 1;
                else if (i > piv && i < w) c[i] = c[i - 1] + 1;
            }
#pragma unroll
            for (int i = 0; i < kWalkMaxW; ++i) {
                if (i >= piv && i <= w - 2) {
#pragma unroll
                    for (int d = 0; d < D; ++d) S[i][d] = (i ? S[i - 1][d] : 0u) ^ s_rows[c[i] * DP + d];
                }
#pragma unroll
                for (int d = 0; d < D; ++d)
                    if (i == w - 2) pre[d] = S[i][d];
                if (i == w - 1) last = c[i];
            }
        }
    }
    const uint32_t wm = wave_min_u32(m);
    const uint64_t ws = wave_sum_u64(done);
    if ((threadIdx.x & 63) == 0) {
        if (wm != kInf) atomicMin(&a.out->min_weight, wm);
        if (ws) atomicAdd((unsigned long long *)&a.out->executed, (unsigned long long)ws);
    }
}

int launch_walk_pair(const WalkArgs &a, int D, int blocks, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (a.k < 1 || a.k > kWalkMaxK || a.w < 1 || a.w > kWalkMaxW || a.w > a.k || blocks < 1) return -2;
    switch (D) {
        case 1: hipLaunchKernelGGL((walk_pair_kernel<1>), dim3(blocks), dim3(256), 0, s, a); break;
        case 2: hipLaunchKernelGGL((walk_pair_kernel<2>), dim3(blocks), dim3(256), 0, s, a); break;
        case 3: hipLaunchKernelGGL((walk_pair_kernel<3>), dim3(blocks), dim3(256), 0, s, a); break;
        case 4: hipLaunchKernelGGL((walk_pair_kernel<4>), dim3(blocks), dim3(256), 0, s, a); break;
        default: return -2;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace md
