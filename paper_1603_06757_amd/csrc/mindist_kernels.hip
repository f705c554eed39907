// mindist_kernels.hip -- gfx950 kernels of the single-code path.
//
// enum_pair_kernel computes, for one pair (Gamma_j, w) of Algorithm 1, the
// least weight of c*Gamma_j over all c with wt(c) = w (the inner minimum of
// Algorithm 1), with the left/right split described in mindist_internal.h.
// Rows and tables are a few KB to a few MB; nothing per codeword touches HBM.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <atomic>

#include "mindist_device.h"

namespace md {

static_assert(sizeof(GroupArgs) <= 4096, "launch arguments exceed the kernel argument space");

template <int D, int B, bool VERIFY, bool MF>
__global__ __launch_bounds__(256) void enum_pair_kernel(GroupArgs ga) {
    const uint64_t t_begin = wall_clock64();
    const int lane = threadIdx.x & 63;
    // this block's pair (blocks of a launch are laid out pair after pair)
    uint32_t g = 0;
    while (g + 1 < ga.n && ga.block_start[g + 1] <= blockIdx.x) ++g;
    g = uni32(g);
    const PairArgs &p = ga.p[g];
    Slot *slots = state_slots(p.st);
    // the least weight this pair may be cut by: the previous launches' and
    // that of pairs 0..g of this launch
    uint32_t *pref = state_prefix_min(p.st, p.max_pairs);
    const uint32_t U_base = uni32(__hip_atomic_load(&p.st->U_base, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT));
    const uint32_t pair_end = ga.p[0].pair + ga.n;
    int gi = 0;
    // per-lane totals over all chunks of this wave, flushed once at the end
    // (per-chunk atomics on the pair record serialise in L2)
    uint32_t run_min = kInf;
    uint64_t run_cnt = 0, run_ws = 0;
    // Wave v runs chunk v first, without a claim; the chunks past the
    // launch's waves go one per claim, so the waves running at the same
    // moment hold neighbouring chunks.  Chunk waves + c is handed out by
    // counter c % nq; a wave starts on counter (v % nq) and moves on, for
    // good, once that counter is past the end.  Counters on separate lines
    // take nq times the claim rate of one.  A pair with no more chunks than
    // waves makes no claim at all.
    const uint32_t nq = p.counters;
    // (readfirstlane: the wave index is uniform, and everything derived from
    // the claimed chunk must stay in scalar registers for the table loads)
    const uint32_t wave = uni32((uint32_t)((blockIdx.x - ga.block_start[g]) * (blockDim.x >> 6) +
                                           (threadIdx.x >> 6)));
    const uint32_t home = wave % nq;
    // binomial columns C(x, a) and C(x, b), x <= k, for the per-lane lookups
    __shared__ uint64_t colA[kBinomX], colB[kBinomX];
    for (int x = threadIdx.x; x <= p.k; x += blockDim.x) {
        colA[x] = binom(p.binom, x, p.a);
        colB[x] = binom(p.binom, x, p.b);
    }
    __syncthreads();
    const ItemSrc src{p.rows, p.table, p.ltable, p.binom, colA, colB, 1, 1,
                      p.n_items, p.k, p.a, p.b, p.b2, p.table2, p.cnt2, kBinomT};
    uint32_t rt_cur = 0;
    uint32_t moved = (uint64_t)p.waves >= p.total_chunks ? nq : 0u;
    bool first = true;
    uint32_t U_seen = kInf;
    for (;;) {
        uint64_t c = 0;
        bool have = false;
        if (first) {
            first = false;
            c = wave;
            have = c < p.total_chunks;
        }
        while (!have && moved < nq) {
            const uint32_t q = (home + moved) % nq;
            uint64_t idx = 0;
            if (lane == 0)
                idx = atomicAdd((unsigned long long *)state_counter(p.st, p.max_pairs, p.pair, q), 1ull);
            idx = uni64((uint64_t)__shfl((long long)idx, 0));
            c = (uint64_t)p.waves + idx * nq + q;
            if (c < p.total_chunks) { have = true; break; }
            ++moved;
        }
        if (!have) break;
        U_seen = min(U_base, uni32(__hip_atomic_load(&pref[p.pair], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)));
        // U at or below the bound before this pair: cut short (a wave of this
        // pair or of an earlier pair of the launch got there), or a pair
        // launched ahead of a run that has ended
        if (p.midpair_exit && U_seen <= p.L_prev) break;
        if (p.cancel_after) {
            uint64_t cl = 0;
            if (lane == 0) cl = atomicAdd((unsigned long long *)&p.st->claimed, 1ull);
            cl = uni64((uint64_t)__shfl((long long)cl, 0));
            if (cl >= p.cancel_after) {
                if (lane == 0) atomicExch(&p.st->cancelled, 1u);
                break;
            }
        }
        ChunkGeo g;
        if (p.order == 0) {
            // left-major: groups of left tiles by the largest element of their
            // first item; a wave's chunk ids grow except when it changes counter
            if (p.groups[gi].chunk_base > c) gi = 0;
            while (gi + 1 < p.ngroups && p.groups[gi + 1].chunk_base <= c) ++gi;
            const GroupEntry ge = p.groups[gi];
            const uint64_t off = c - ge.chunk_base;
            g.lt = ge.lt_begin + off / ge.n_rt;
            const uint32_t rt = (uint32_t)(off % ge.n_rt);
            g.i_begin = rt * p.T;
            g.i_end = min(g.i_begin + p.T, ge.nr_first);
            g.e_first = ge.e;
            g.clip = false;
        } else {
            // right-major: right tile r holds the left tiles whose first item
            // still has entries past r*T; find r by binary search
            uint32_t lo = (p.rprefix[rt_cur] <= c) ? rt_cur : 0u, hi = p.n_rt - 1;
            while (lo < hi) {
                const uint32_t mid = (lo + hi + 1) >> 1;
                if (p.rprefix[mid] <= c) lo = mid; else hi = mid - 1;
            }
            rt_cur = lo;
            g.lt = c - p.rprefix[lo];
            g.i_begin = lo * p.T;
            g.i_end = g.i_begin + p.T;
            g.e_first = 0;
            g.clip = true;
        }
        uint32_t L[B][D], nr[B], lmin, ws;
        uint64_t cnt;
        if (p.b2) run_chunk3<D, B, VERIFY>(src, g, L, nr, lmin, cnt, ws);
        else run_chunk<D, B, VERIFY, MF ? 2 : 0>(src, g, L, nr, lmin, cnt, ws);
        run_min = min(run_min, lmin);
        run_cnt += cnt;
        if (VERIFY) run_ws += ws;
        // only a lane that beats U (as last read) takes part in the update
        const bool better = lmin != kInf && lmin + p.offset < U_seen;
        if (!__ballot(better)) continue;
        const uint32_t wmin = wave_min_u32(lmin);
        const uint32_t val = wmin + p.offset;
        uint32_t old = 0;
        if (lane == 0) {
            old = atomicMin(&p.st->U_found, val);
            for (uint32_t q = p.pair; q < pair_end; ++q) atomicMin(&pref[q], val);
        }
        old = uni32((uint32_t)__shfl((int)old, 0));
        U_seen = min(U_seen, val);
        if (old > val) {
            // this wave moved U_found to val: it alone writes slot[val]
            uint32_t hit_i, hit_i2 = 0;
            uint64_t hit_rho;
            const int first = p.b2 ? find_witness3<D, B>(src, g, L, nr, wmin, hit_i, hit_i2, hit_rho)
                                   : find_witness<D, B>(src, g, L, nr, wmin, hit_i, hit_rho);
            if (lane == first) {
                slots[val].pair = p.pair;
                slots[val].i = hit_i;
                slots[val].i2 = hit_i2;
                slots[val].rho = hit_rho;
            }
        }
        if (p.midpair_exit && val <= p.L_prev && lane == 0)
            __hip_atomic_store(&p.st->exit_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const uint32_t wmin = wave_min_u32(run_min);
    const uint64_t wcnt = wave_sum_u64(run_cnt);
    const uint64_t wws = VERIFY ? wave_sum_u64(run_ws) : 0ull;
    if (lane == 0) {
        WavePart *wp = p.parts + wave;
        wp->pair_min = wmin == kInf ? kInf : wmin + p.offset;
        wp->executed = wcnt;
        wp->wsum = VERIFY ? wws + (uint64_t)p.offset * wcnt : 0ull;
        wp->t0 = t_begin;
        wp->t1 = wall_clock64();
    }
}

// Runs right behind a launch (stream order makes every wave's totals and the
// run state visible): one block reduces each pair's waves' totals and
// publishes them with the run state to the pair's pinned mailbox, sequence
// word last; then records U_found as the next launch's U_base.
__global__ __launch_bounds__(1024) void publish_pair_kernel(GroupArgs ga, PairMail *mails) {
    __shared__ uint32_t s_mn[16];
    __shared__ uint64_t s_ex[16], s_ws[16], s_t0[16], s_t1[16];
    __shared__ uint32_t r_mn[kGroupMax];
    __shared__ uint64_t r_ex[kGroupMax], r_ws[kGroupMax], r_t0[kGroupMax], r_t1[kGroupMax];
    DevState *st = ga.p[0].st;
    const int lane = threadIdx.x & 63;
    const uint32_t nwv = blockDim.x >> 6, wv = threadIdx.x >> 6, n = ga.n;
    // wave wv reduces pair wv % n (every pair gets nwv / n waves or one more,
    // all pairs at once), over its entries lane + 64 * (wv / n + k * per)
    {
        const uint32_t g = wv % n;
        const uint32_t per = (nwv - g + n - 1) / n;    // waves on pair g
        const PairArgs &p = ga.p[g];
        uint32_t mn = kInf;
        uint64_t ex = 0, ws = 0, t0 = ~0ull, t1 = 0;
        for (uint32_t v = lane + 64u * (wv / n); v < p.waves; v += 64u * per) {
            mn = min(mn, p.parts[v].pair_min);
            ex += p.parts[v].executed;
            ws += p.parts[v].wsum;
            t0 = min(t0, p.parts[v].t0);
            t1 = max(t1, p.parts[v].t1);
        }
        mn = wave_min_u32(mn);
        ex = wave_sum_u64(ex);
        ws = wave_sum_u64(ws);
        t0 = wave_min_u64(t0);
        t1 = wave_max_u64(t1);
        if (lane == 0) {
            s_mn[wv] = mn;
            s_ex[wv] = ex;
            s_ws[wv] = ws;
            s_t0[wv] = t0;
            s_t1[wv] = t1;
        }
    }
    __syncthreads();
    if (threadIdx.x < n) {
        const uint32_t g = threadIdx.x;
        uint32_t mn = kInf;
        uint64_t ex = 0, ws = 0, t0 = ~0ull, t1 = 0;
        for (uint32_t w = g; w < nwv; w += n) {
            mn = min(mn, s_mn[w]);
            ex += s_ex[w];
            ws += s_ws[w];
            t0 = min(t0, s_t0[w]);
            t1 = max(t1, s_t1[w]);
        }
        r_mn[g] = mn;
        r_ex[g] = ex;
        r_ws[g] = ws;
        r_t0[g] = t0;
        r_t1[g] = t1;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    // the run state, the same for every pair of the launch
    const uint32_t U = __hip_atomic_load(&st->U_found, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t exit_flag = __hip_atomic_load(&st->exit_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t cancelled = __hip_atomic_load(&st->cancelled, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    Slot wit{};
    if (U <= kMaxSlot) wit = state_slots(st)[U];
    for (uint32_t g = 0; g < ga.n; ++g) {
        PairMail *m = mails + ga.p[g].pair % kMailRing;
        m->t_begin = r_t0[g];
        m->t_end = r_t1[g];
        m->U_found = U;
        if (U <= kMaxSlot) m->witness = wit;
        m->exit_flag = exit_flag;
        m->cancelled = cancelled;
        m->pair_min = r_mn[g];
        m->executed = r_ex[g];
        m->wsum = r_ws[g];
    }
    // every mailbox's contents before any sequence word: one system fence,
    // then relaxed stores (a release store would repeat the L2 write-back
    // of the fence for every mailbox)
    __threadfence_system();
    for (uint32_t g = 0; g < ga.n; ++g)
        __hip_atomic_store(&mails[ga.p[g].pair % kMailRing].seq, ga.p[g].pair + 1, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&st->U_base, U, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Calibration: the hot loop of enum_pair_kernel with nothing around it.
// Every lane holds B left sums, the wave walks a 64-entry right table (kept
// in the scalar cache) for `steps` entries per pass; no unranking, no
// tails, no atomics.  Its rate is the ceiling of the enumeration's
// instruction mix on this device and clock.
template <int D, int B>
__global__ __launch_bounds__(256) void peak_xorpop_kernel(const uint32_t *tab, uint32_t steps,
                                                          uint32_t *out) {
    uint32_t L[B][D], nr[B], vm[B], m[B];
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int t = 0; t < B; ++t) {
#pragma unroll
        for (int d = 0; d < D; ++d) L[t][d] = gid * 0x9E3779B9u + (uint32_t)(t * 7 + d) * 0x85EBCA6Bu;
        nr[t] = kInf;
        vm[t] = kInf;
        m[t] = kInf;
    }
    uint32_t ws = 0;
    for (uint32_t i = 0; i < steps; i += 64)
        run_range<D, B, false, false>(tab, 0, 64, L, nr, vm, m, ws);
    uint32_t r = kInf;
#pragma unroll
    for (int t = 0; t < B; ++t) r = min(r, m[t]);
    if (r == 0x12345678u) out[gid] = r;    // keeps the loop alive
}

int launch_peak(const uint32_t *tab, uint32_t steps, uint32_t *out, int D, int blocks, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    switch (D) {
        case 1: hipLaunchKernelGGL((peak_xorpop_kernel<1, 4>), dim3(blocks), dim3(256), 0, s, tab, steps, out); break;
        case 2: hipLaunchKernelGGL((peak_xorpop_kernel<2, 4>), dim3(blocks), dim3(256), 0, s, tab, steps, out); break;
        case 3: hipLaunchKernelGGL((peak_xorpop_kernel<3, 4>), dim3(blocks), dim3(256), 0, s, tab, steps, out); break;
        case 4: hipLaunchKernelGGL((peak_xorpop_kernel<4, 4>), dim3(blocks), dim3(256), 0, s, tab, steps, out); break;
        case 7: hipLaunchKernelGGL((peak_xorpop_kernel<7, 4>), dim3(blocks), dim3(256), 0, s, tab, steps, out); break;
        case 8: hipLaunchKernelGGL((peak_xorpop_kernel<8, 4>), dim3(blocks), dim3(256), 0, s, tab, steps, out); break;
        default: return -2;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Register-only ceiling of the enumeration's arithmetic: every lane holds
// B x D 32-bit words; per step the wave XORs them with D wave-uniform words
// (scalar registers, new every step) and accumulates their popcounts, one
// v_xor_b32 + one v_bcnt_u32_b32 per word, into B independent chains; U
// steps per loop iteration.  No memory operation inside the loop.
// ops = grid threads x steps x B x D.
template <int B, int D, int U>
__global__ __launch_bounds__(256) void peak_reg_kernel(uint32_t steps, uint32_t seed, uint32_t *out) {
    uint32_t L[B][D], acc[B];
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
    for (int t = 0; t < B; ++t) {
#pragma unroll
        for (int d = 0; d < D; ++d) L[t][d] = (gid + 1) * 0x9E3779B9u ^ (uint32_t)(t * D + d) * 0x85EBCA6Bu;
        acc[t] = 0;
    }
    for (uint32_t i = 0; i < steps; i += U) {
        const uint32_t s = uni32(seed ^ (i * 0x27D4EB2Fu));
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const uint32_t sd = s + (uint32_t)(u * D + d) * 0x165667B1u;
#pragma unroll
                for (int t = 0; t < B; ++t) acc[t] = bcnt_acc(L[t][d] ^ sd, acc[t]);
            }
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int t = 0; t < B; ++t) r += acc[t];
    out[gid] = r;              // every lane stores its sum: the chains stay live
}

// variant v: (lane items, words, steps per iteration)
int peak_reg_shape(int v, int *items, int *words) {
    static const int shape[kPeakVariants][2] = {{8, 4}, {8, 4}, {4, 6}, {16, 2}};
    if (v < 0 || v >= kPeakVariants) return -1;
    *items = shape[v][0];
    *words = shape[v][1];
    return 0;
}

int launch_peak_reg(int v, uint32_t steps, uint32_t seed, uint32_t *out, int blocks, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    switch (v) {
        case 0: hipLaunchKernelGGL((peak_reg_kernel<8, 4, 1>), dim3(blocks), dim3(256), 0, s, steps, seed, out); break;
        case 1: hipLaunchKernelGGL((peak_reg_kernel<8, 4, 4>), dim3(blocks), dim3(256), 0, s, steps, seed, out); break;
        case 2: hipLaunchKernelGGL((peak_reg_kernel<4, 6, 4>), dim3(blocks), dim3(256), 0, s, steps, seed, out); break;
        case 3: hipLaunchKernelGGL((peak_reg_kernel<16, 2, 4>), dim3(blocks), dim3(256), 0, s, steps, seed, out); break;
        default: return -2;
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Saved sums (see TableArgs): entry i = rows of colex_unrank_b(i) (left) or
// rows {k-1-shift-z} (right / outer); outer tables also record the number of
// inner entries C(shift + min z, shift) above each entry.
template <int D>
__global__ __launch_bounds__(256) void build_table_kernel(TableArgs ta) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ta.entries) return;
    uint32_t acc[D];
#pragma unroll
    for (int d = 0; d < D; ++d) acc[d] = 0;
    uint64_t rho = i;
    int hi = ta.k - ta.shift, zmin = 0;
    for (int t = ta.b; t >= 1; --t) {
        int lo = t - 1, h = hi - 1;
        while (lo < h) {
            const int mid = (lo + h + 1) >> 1;
            if (binom(ta.binom, mid, t) <= rho) lo = mid; else h = mid - 1;
        }
        rho -= binom(ta.binom, lo, t);
        hi = lo;
        zmin = lo;
        const int r = ta.reflect ? (ta.k - 1 - ta.shift - lo) : lo;
#pragma unroll
        for (int d = 0; d < D; ++d) acc[d] ^= ta.rows[(size_t)r * ta.dp + d];
    }
#pragma unroll
    for (int d = 0; d < D; ++d) ta.table[i * ta.dp + d] = acc[d];
    for (int d = D; d < ta.dp; ++d) ta.table[i * ta.dp + d] = 0;
    if (ta.cnt2) ta.cnt2[i] = (uint32_t)binom(ta.binom, ta.shift + zmin, ta.shift);
}

// Level b from level b-1 (TableArgs::prev): one search of the block of
// the entry's largest element in LDS, one row and one lower-level entry.
template <int D>
__global__ __launch_bounds__(256) void extend_table_kernel(TableArgs ta) {
    __shared__ uint64_t start[kBinomX];      // start[m] = C(m, b): first entry of block m
    for (int x = threadIdx.x; x <= ta.k; x += blockDim.x) start[x] = binom(ta.binom, x, ta.b);
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ta.entries) return;
    int lo = ta.b - 1, hi = ta.k - 1;          // largest m with C(m, b) <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= i) lo = mid; else hi = mid - 1;
    }
    const uint64_t r = i - start[lo];
    const int row = ta.reflect ? (ta.k - 1 - lo) : lo;
#pragma unroll
    for (int d = 0; d < D; ++d)
        ta.table[i * ta.dp + d] = ta.rows[(size_t)row * ta.dp + d] ^ ta.prev[r * ta.dp + d];
    for (int d = D; d < ta.dp; ++d) ta.table[i * ta.dp + d] = 0;
}

__global__ void init_state_kernel(DevState *st, int max_pairs) {
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    for (int q = tid; q < max_pairs * kCounters; q += gridDim.x * blockDim.x)
        *state_counter(st, max_pairs, q / kCounters, q % kCounters) = 0;
    if (tid == 0) {
        st->U_found = kInf;
        st->exit_flag = 0;
        st->cancelled = 0;
        st->U_base = kInf;
        st->claimed = 0;
    }
    uint32_t *pref = state_prefix_min(st, max_pairs);
    for (int q = tid; q < max_pairs; q += gridDim.x * blockDim.x) pref[q] = kInf;
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, uint64_t count) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------------------
int max_dwords() { return 16; }

int launch_fill_u32(uint32_t *p, uint32_t v, uint64_t count, void *stream) {
    if (!count) return 0;
    const uint64_t blocks = std::min<uint64_t>((count + 255) / 256, 1024);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, p, v,
                       count);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

static int check(hipError_t e) { return e == hipSuccess ? 0 : -1; }

int launch_init_state(DevState *st, int max_pairs, void *stream) {
    hipLaunchKernelGGL(init_state_kernel, dim3(64), dim3(256), 0, (hipStream_t)stream, st,
                       max_pairs);
    return check(hipGetLastError());
}

template <int D>
static void table_launch(const TableArgs &ta, hipStream_t s) {
    const uint64_t blocks = (ta.entries + 255) / 256;
    if (ta.prev)
        hipLaunchKernelGGL(extend_table_kernel<D>, dim3((unsigned)blocks), dim3(256), 0, s, ta);
    else
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

template <int D, int B>
static void enum_launch_b(const GroupArgs &ga, int verify, int mfma, int blocks, hipStream_t s) {
    if (verify)
        hipLaunchKernelGGL((enum_pair_kernel<D, B, true, false>), dim3(blocks), dim3(256), 0, s, ga);
    else if constexpr (D <= kMfmaMaxD) {
        if (mfma)
            hipLaunchKernelGGL((enum_pair_kernel<D, B, false, true>), dim3(blocks), dim3(256), 0, s, ga);
        else
            hipLaunchKernelGGL((enum_pair_kernel<D, B, false, false>), dim3(blocks), dim3(256), 0, s, ga);
    } else {
        hipLaunchKernelGGL((enum_pair_kernel<D, B, false, false>), dim3(blocks), dim3(256), 0, s, ga);
    }
}

template <int D>
static void enum_launch(const GroupArgs &ga, int items, int verify, int mfma, int blocks, hipStream_t s) {
    if (items == 4) enum_launch_b<D, 4>(ga, verify, mfma, blocks, s);
    else enum_launch_b<D, 2>(ga, verify, mfma, blocks, s);
}

template <int D, int B>
static int mfma_resident() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, enum_pair_kernel<D, B, false, true>, 256, 0) !=
        hipSuccess)
        return 0;
    return n;
}

int enum_mfma_resident_blocks(int D, int items) {
    // the answer depends only on the kernel's resources: asked once per shape
    static std::atomic<int> cache[kMfmaMaxD + 1][2];
    if (D < 1 || D > kMfmaMaxD || (items != 2 && items != 4)) return 0;
    std::atomic<int> &slot = cache[D][items == 4];
    int n = slot.load(std::memory_order_relaxed);
    if (n > 0) return n;
    switch (D * 8 + items) {
        case 1 * 8 + 2: n = mfma_resident<1, 2>(); break;
        case 1 * 8 + 4: n = mfma_resident<1, 4>(); break;
        case 2 * 8 + 2: n = mfma_resident<2, 2>(); break;
        case 2 * 8 + 4: n = mfma_resident<2, 4>(); break;
        case 3 * 8 + 2: n = mfma_resident<3, 2>(); break;
        case 3 * 8 + 4: n = mfma_resident<3, 4>(); break;
        case 4 * 8 + 2: n = mfma_resident<4, 2>(); break;
        case 4 * 8 + 4: n = mfma_resident<4, 4>(); break;
        default: break;
    }
    if (n > 0) slot.store(n, std::memory_order_relaxed);
    return n;
}

int launch_publish_pair(const GroupArgs &ga, PairMail *mail, void *stream) {
    hipLaunchKernelGGL(publish_pair_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, ga, mail);
    return check(hipGetLastError());
}

int launch_enum_pair(const GroupArgs &ga, int D, int items, int verify, int mfma, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    if (ga.n < 1 || ga.n > (uint32_t)kGroupMax || ga.block_start[0] != 0) return -1;
    for (uint32_t g = 0; g < ga.n; ++g)
        if (ga.block_start[g + 1] <= ga.block_start[g] || ga.p[g].pair != ga.p[0].pair + g ||
            ga.p[g].waves != 4u * (ga.block_start[g + 1] - ga.block_start[g]))
            return -1;
    const int blocks = (int)ga.block_start[ga.n];
    switch (D) {
#define MD_CASE(X) case X: enum_launch<X>(ga, items, verify, mfma, blocks, s); break;
        MD_CASE(1) MD_CASE(2) MD_CASE(3) MD_CASE(4) MD_CASE(5) MD_CASE(6) MD_CASE(7) MD_CASE(8)
        MD_CASE(9) MD_CASE(10) MD_CASE(11) MD_CASE(12) MD_CASE(13) MD_CASE(14) MD_CASE(15)
        MD_CASE(16)
#undef MD_CASE
        default: return -2;
    }
    return check(hipGetLastError());
}

}  // namespace md
