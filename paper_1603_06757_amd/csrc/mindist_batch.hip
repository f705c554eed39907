// mindist_batch.hip -- the persistent multi-code kernel (see mindist_batch.h).
//
// Waves walk the code slots, claim one chunk at a time from a code's open
// job (spread over the job's counters) and stay on that code while it has
// chunks; a wave adds its completed chunks to the job once, when it finds
// the job drained.  Jobs:
//   * table job: the code's saved right sums (Section 3.4), 4096 entries per
//     chunk;
//   * pair (Gamma_j, w): the same left/right enumeration as the single-code
//     kernel (two left subsets per lane, left subsets unranked per lane).
// The wave that completes a job's last chunk applies Algorithm 1's control
// for that code: L after the pair (one raise per Gamma_j), the test L >= U,
// and opens the next pair or marks the code done.
#include <hip/hip_runtime.h>

#include "mindist_batch.h"
#include "mindist_device.h"

namespace md {
namespace {

__device__ __forceinline__ uint32_t ld_acq(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_acq(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_acq(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_rlx(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Coherent reads of what another wave published during the launch (job
// records, chunk groups): device-scope loads see the data the publishing
// wave released, with no cache-wide invalidation.  Each XCD has its own L2:
// an acquire fence at device scope invalidates the reading XCD's whole L2,
// which the waves' table reads then pay for; the job's address comes from
// the published offset, so these loads follow the publication.
__device__ __forceinline__ uint32_t ldc(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ldc(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ldc(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(int32_t *p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// lane 0 does the atomic, every lane gets the (uniform) result
__device__ __forceinline__ uint64_t wave_fetch_add(uint64_t *p, uint64_t v) {
    uint64_t r = 0;
    if ((threadIdx.x & 63) == 0) r = atomicAdd((unsigned long long *)p, (unsigned long long)v);
    return uni64((uint64_t)__shfl((long long)r, 0));
}

// counters for a job of `total` chunks: one per 64 chunks, at most kJobCounters
__device__ __forceinline__ uint32_t job_counters(uint64_t total) {
    const uint64_t c = total / 64;
    return c < 1 ? 1u : (c > (uint64_t)kJobCounters ? (uint32_t)kJobCounters : (uint32_t)c);
}

__device__ __forceinline__ GroupEntry *job_groups(BatchJob *jb) {
    return reinterpret_cast<GroupEntry *>(jb + 1);
}
__device__ __forceinline__ BatchJob *job_at(const BatchArgs &A, uint32_t off) {
    return reinterpret_cast<BatchJob *>(A.arena + (size_t)off * 128);
}

__device__ int bound_f_dev(int i, int h, int m_full, int k, int k_m) {
    if (i < m_full) return h + 1;
    const int v = h + 1 - (k - k_m);
    return v > 0 ? v : 0;
}
// L after pair (j, w): one raise per Gamma_j (Section 2)
__device__ int bound_after_dev(int k, int m_full, int k_m, int ng, int j, int w) {
    int s = 0;
    for (int i = 0; i < ng; ++i) s += bound_f_dev(i, i <= j ? w : w - 1, m_full, k, k_m);
    return s;
}

// Allocate a job record with room for `ngroups_cap` group entries; returns
// its arena offset or 0xFFFFFFFF when the arena is full.
__device__ uint32_t alloc_job(const BatchArgs &A, int c, int ngroups_cap) {
    const uint64_t bytes = sizeof(BatchJob) + sizeof(GroupEntry) * (uint64_t)ngroups_cap;
    const uint64_t units = (bytes + 127) / 128;
    if (A.serving) {              // the code's own segment (reset when its slot is reused)
        BatchCode *cs = &A.codes[c];
        const uint64_t off = wave_fetch_add(&cs->arena_next, units);
        if (off + units > cs->arena_hi || off + units > 0xFFFFFFFFull) return 0xFFFFFFFFu;
        return (uint32_t)off;
    }
    const uint64_t off = wave_fetch_add(&A.g->arena_next, units);
    if (off + units > A.g->arena_cap || off + units > 0xFFFFFFFFull) return 0xFFFFFFFFu;
    return (uint32_t)off;
}

// Serving: copy what the host needs to decode code c into its mirror in
// pinned host memory (16-byte stores spread over the wave's lanes).
__device__ __noinline__ void mirror_code(const BatchArgs &A, int c) {
    const int lane = threadIdx.x & 63;
    const BatchCode *cs = &A.codes[c];
    ServeMirror *m = A.mirror + c;
    const uint4 *src = reinterpret_cast<const uint4 *>(cs);
    uint4 *dst = reinterpret_cast<uint4 *>(m->code);
    for (int q = lane; q < (int)(sizeof(m->code) / 16); q += 64) dst[q] = src[q];
    const int nj = cs->njobs < kBatchMaxPairs ? cs->njobs : kBatchMaxPairs;
    for (int q = lane; q < nj * 8; q += 64) {
        const uint4 *jl = reinterpret_cast<const uint4 *>(job_at(A, cs->job[q >> 3]));
        reinterpret_cast<uint4 *>(m->jobs[q >> 3])[q & 7] = jl[q & 7];
    }
    const uint32_t u = cs->U_found;
    if (u != kInf && u <= (uint32_t)cs->n && lane < 2)
        reinterpret_cast<uint4 *>(&m->witness)[lane] = reinterpret_cast<const uint4 *>(&cs->slots[u])[lane];
}

__device__ __noinline__ void finish_code(const BatchArgs &A, int c, int32_t status, uint32_t L, uint32_t U) {
    BatchCode *cs = &A.codes[c];
    const int lane = threadIdx.x & 63;
    if (lane == 0) {
        cs->L_final = L;
        cs->U_final = U;
        cs->t_done = wall_clock64();
    }
    __threadfence();
    if (lane == 0) {
        st_rel(&cs->status, status);
        atomicAdd(&A.g->codes_done, 1u);
    }
    if (A.host_done) {
        __threadfence();
        if (A.mirror) mirror_code(A, c);
        __threadfence_system();
        if (lane == 0)
            __hip_atomic_store(&A.host_done[c], (uint32_t)cs->seq, __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

// Open pair (j, w) as job p of code c (whole wave).  Mirrors the host's
// plan: b = min(w/2, bcap_j), a = w - b, left tiles of 64*batch_items(D_j)
// subsets grouped by the largest element e of their first subset.
__device__ void open_pair(const BatchArgs &A, int c, int p, int j, int w, uint32_t L_before) {
    BatchCode *cs = &A.codes[c];
    const int lane = threadIdx.x & 63;
    const int k = cs->k;
    const BatchSet &set = cs->sets[j];
    // split: the rule of the host planner, with the inner size fixed to
    // bcap, the shift the outer tables were built with
    int a, b, b2;
    split_rows(k, w, set.bcap, true, [&](int x, int r) { return binom(A.binom, x, r); }, a, b, b2);
    const uint64_t TB = 64ull * batch_items(set.D);
    const uint64_t n_items = binom(A.binom, k - b - b2, a);
    const uint64_t tiles = (n_items + TB - 1) / TB;
    // The waves this pair can expect are the launch's waves over the codes
    // still running (the chunks-per-visit quantum spreads them); it should
    // leave each of them max(2, D-1) chunks.
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x >> 6);
    const uint32_t done = uni32(ld_rlx(&A.g->codes_done));
    const uint32_t l0 = uni32(ld_rlx(&A.g->live0));
    const uint32_t live0 = l0 ? l0 : (uint32_t)A.n_codes;
    const uint64_t live = live0 > done ? (uint64_t)(live0 - done) : 1ull;
    const uint64_t share = waves / live > 0 ? waves / live : 1ull;
    const uint64_t need = (uint64_t)(set.D > 3 ? set.D - 1 : 2) * share;
    uint32_t T;
    if (b2 == 0) {
        // Right tile from the exact chunk count at each length 16 << t: a
        // left tile whose first subset has largest element e meets
        // C(k-1-e, b) right entries.  From the lower configured bound, longer
        // while the chunks allow (short codes' per-chunk set-up dominates
        // below that bound; long pairs gain from long tiles).  Few live
        // codes (a batch's heavy tail, a code served alone): shorter than
        // the bound where the pair is short, so it is not a few long tiles
        // walked by a few waves while the rest wait for its next pair.
        constexpr int kCand = 10;                // T = 16 .. 8192
        uint64_t ch[kCand];
        for (int t = 0; t < kCand; ++t) ch[t] = 0;
        for (int e0 = a - 1; e0 <= k - 1 - b; e0 += 64) {
            const int e = e0 + lane;
            uint64_t nlt = 0, nr = 0;
            if (e <= k - 1 - b) {
                const uint64_t lt_lo = (binom(A.binom, e, a) + TB - 1) / TB;
                uint64_t lt_hi = (binom(A.binom, e + 1, a) + TB - 1) / TB;
                if (lt_hi > tiles) lt_hi = tiles;
                if (lt_hi > lt_lo) {
                    nlt = lt_hi - lt_lo;
                    nr = binom(A.binom, k - 1 - e, b);
                }
            }
#pragma unroll
            for (int t = 0; t < kCand; ++t) ch[t] += wave_sum_u64(nlt * ((nr + (16ull << t) - 1) >> (4 + t)));
        }
        auto chunks_at = [&](uint32_t TT) {
            uint64_t r = 0;
#pragma unroll
            for (int t = 0; t < kCand; ++t)
                if ((16u << t) == TT) r = ch[t];
            return r;
        };
        const uint32_t t_hi = min(min(A.tile_max, cs->tile_cap), 8192u);
        T = min(A.tile_min, t_hi);
        if (chunks_at(T) >= need) {
            while (T < t_hi && chunks_at(T << 1) >= need) T <<= 1;
        } else if (share >= 16) {
            while (T > 16 && chunks_at(T) < need) T >>= 1;
        }
    } else {
        // outer tile: about 256K codewords per chunk; with at most 4 live
        // codes, the pair's share per expected chunk, down to 4K (a pair of
        // 10^7 codewords would otherwise be 40 chunks: 40 waves, each alone
        // on its CU with nothing to hide its loads behind, ~3 ms instead of
        // ~0.3-0.6 ms; with more live codes the smaller chunks cost more
        // than they spread)
        const int e = (k - b - b2) * a / (a + 1);
        const uint64_t outer = binom(A.binom, k - 1 - b2 - e, b);
        const uint64_t both = binom(A.binom, k - 1 - e, b + b2);
        const double n2 = outer ? (double)both / (double)outer : 1.0;
        double target = 262144.0;
        if (share >= waves / 4) {
            const double fair = (double)binom(A.binom, k, w) / (double)need;
            if (fair < target) target = fair > 4096.0 ? fair : 4096.0;
        }
        const double want = target / ((double)TB * (n2 > 1 ? n2 : 1));
        T = 1;
        while (T < 1024 && T * 2 <= want) T <<= 1;
    }
    const uint32_t off = alloc_job(A, c, k + 2);
    if (off == 0xFFFFFFFFu) {
        finish_code(A, c, -5 /* MINDIST_E_LIMIT */, L_before, min(uni32(ldc(&cs->U_found)), (uint32_t)(cs->n - k + 1)));
        return;
    }
    BatchJob *jb = job_at(A, off);
    GroupEntry *gr = job_groups(jb);
    // groups: one lane per candidate e, compacted with wave prefix sums
    const int e_lo = a - 1, e_hi = k - 1 - b - b2;
    uint64_t chunk_base = 0;
    uint32_t ng = 0;
    for (int e0 = e_lo; e0 <= e_hi; e0 += 64) {
        const int e = e0 + lane;
        uint64_t chunks = 0, lt_lo = 0;
        uint32_t nr_first = 0;
        uint64_t n_rt = 0;
        if (e <= e_hi) {
            const uint64_t lo = binom(A.binom, e, a), hi = binom(A.binom, e + 1, a);
            lt_lo = (lo + TB - 1) / TB;
            uint64_t lt_hi = (hi + TB - 1) / TB;
            if (lt_hi > tiles) lt_hi = tiles;
            if (lt_hi > lt_lo) {
                nr_first = (uint32_t)binom(A.binom, k - 1 - b2 - e, b);
                n_rt = (nr_first + T - 1) / T;
                chunks = (lt_hi - lt_lo) * n_rt;
            }
        }
        const bool has = chunks > 0;
        // exclusive prefix over lanes of (has) and (chunks)
        uint64_t inc_c = chunks;
        uint32_t inc_n = has ? 1u : 0u;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint64_t yc = (uint64_t)__shfl_up((long long)inc_c, o);
            const uint32_t yn = (uint32_t)__shfl_up((int)inc_n, o);
            if (lane >= o) { inc_c += yc; inc_n += yn; }
        }
        if (has) {
            GroupEntry &ge = gr[ng + inc_n - 1];
            ge.chunk_base = chunk_base + inc_c - chunks;
            ge.lt_begin = lt_lo;
            ge.n_rt = n_rt;
            ge.nr_first = nr_first;
            ge.e = (uint32_t)e;
        }
        chunk_base += uni64((uint64_t)__shfl((long long)inc_c, 63));
        ng += uni32((uint32_t)__shfl((int)inc_n, 63));
    }
    if (chunk_base == 0) {        // cannot happen for w <= k; never leave a job nobody can close
        finish_code(A, c, -4 /* MINDIST_E_HIP */, L_before, min(uni32(ldc(&cs->U_found)), (uint32_t)(cs->n - k + 1)));
        return;
    }
    if (lane == 0) {
        jb->kind = 1;
        jb->j = j;
        jb->w = w;
        jb->a = a;
        jb->b = b;
        jb->b2 = b2;
        jb->T = T;
        jb->L_before = L_before;
        jb->offset = set.stripped ? (uint32_t)w : 0u;
        jb->ngroups = ng;
        jb->n_items = n_items;
        jb->total_chunks = chunk_base;
        jb->count = binom(A.binom, k, w);
        jb->pair_min = kInf;
        jb->exit_flag = 0;
        jb->L_after = 0;
        jb->U_after = 0;
        jb->executed = 0;
        jb->expected = chunk_base;
        jb->t_open = wall_clock64();
        jb->t_close = 0;
        jb->nctr = job_counters(chunk_base);
        for (int r = 0; r < kJobCounters; ++r) jb->claim[r].v = 0;
        jb->done = 0;
        jb->drained_mask = 0;
        cs->job[p] = off;
    }
    // the group entries of every lane and the record, then the job count:
    // the lanes' stores complete, lane 0's release writes them back
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) st_rel(&cs->njobs, p + 1);
}

// The table job (job 0): every right table of every set of the code.
__device__ void open_tables(const BatchArgs &A, int c) {
    BatchCode *cs = &A.codes[c];
    const uint32_t off = alloc_job(A, c, 0);
    if (off == 0xFFFFFFFFu) {
        finish_code(A, c, -5, 1, (uint32_t)(cs->n - cs->k + 1));
        return;
    }
    BatchJob *jb = job_at(A, off);
    if ((threadIdx.x & 63) == 0) {
        const uint64_t E = cs->tab_off[kBatchTabs];
        cs->t_open = wall_clock64();
        jb->kind = 0;
        jb->j = -1;
        // chunks of kTableChunk entries, halved (down to kTableChunkMin) while
        // that leaves fewer than kTableChunksWanted of them: a short code's
        // tables are a few thousand entries, built by as many waves
        uint32_t tc = kTableChunk;
        while (tc > kTableChunkMin && (E + tc - 1) / tc < kTableChunksWanted) tc >>= 1;
        jb->T = tc;
        jb->total_chunks = (E + tc - 1) / tc;
        jb->expected = jb->total_chunks;
        jb->t_open = wall_clock64();
        jb->t_close = 0;
        jb->nctr = job_counters(jb->total_chunks);
        for (int r = 0; r < kJobCounters; ++r) jb->claim[r].v = 0;
        jb->done = 0;
        jb->drained_mask = 0;
        jb->executed = 0;
        jb->pair_min = kInf;
        cs->job[0] = off;
    }
    __threadfence();
    if ((threadIdx.x & 63) == 0) {
        st_rel(&cs->njobs, 1);
        st_rel(&cs->status, (int32_t)kSlotActive);
    }
}

// n consecutive entries of one saved table of level BL, from entry i on:
// the first by unranking, the rest by the colex successor (one or two row
// additions each).  Entry e is the sum of rows {kk-1-z : z in
// colex_unrank_BL(e)}; an outer table (cnt != nullptr, rows [0, kk) with
// kk = k - shift) also stores C(shift + min z, shift), the inner count.
// BL is a template parameter so that the subset stays in registers; the run
// is not inlined so that it does not set the persistent kernel's register
// budget.  The binomials come from the block's LDS slice, C(x, t) at
// bt[x * kLdsBinomT + t] (x < 256, t <= 8 covers every run of a code of the
// batch layout: k <= 256, BL and the shift <= kBatchMaxB), so that the first
// entry's unranking and an outer table's inner counts are not chains of
// global loads.
typedef __attribute__((address_space(3))) const uint64_t LdsU64;
template <int BL>
__device__ __noinline__ void table_run(LdsU64 *bt, const uint32_t *rows, int dp, int D,
                                          int kk, int shift, uint32_t *out, uint32_t *cnt,
                                          uint64_t i, uint64_t n) {
    auto C = [&](int x, int t) { return (x < 0 || t < 0 || t > x) ? 0ull : bt[x * kLdsBinomT + t]; };
    int z[BL + 1];
    uint32_t acc[kBatchMaxD];
#pragma unroll
    for (int d = 0; d < kBatchMaxD; ++d) acc[d] = 0;
    auto add_row = [&](int zz) {
        const uint32_t *row = rows + (size_t)(kk - 1 - zz) * dp;
#pragma unroll
        for (int d = 0; d < kBatchMaxD; ++d)
            if (d < D) acc[d] ^= row[d];
    };
    {
        uint64_t r = i;
        int top = kk;
#pragma unroll
        for (int t = BL; t >= 1; --t) {
            int l = t - 1, h = top - 1;
            while (l < h) {
                const int mid = (l + h + 1) >> 1;
                if (C(mid, t) <= r) l = mid; else h = mid - 1;
            }
            r -= C(l, t);
            top = l;
            z[t - 1] = l;
            add_row(l);
        }
    }
    z[BL] = kk;                       // sentinel
    for (uint64_t e = 0; e < n; ++e, ++i) {
        uint32_t *o = out + (size_t)i * dp;
        if (dp == 8) {
            *reinterpret_cast<uint4 *>(o) = make_uint4(acc[0], acc[1], acc[2], acc[3]);
            *reinterpret_cast<uint4 *>(o + 4) = make_uint4(acc[4], acc[5], acc[6], acc[7]);
        } else if (dp == 4) {
            *reinterpret_cast<uint4 *>(o) = make_uint4(acc[0], acc[1], acc[2], acc[3]);
        } else if (dp == 2) {
            *reinterpret_cast<uint2 *>(o) = make_uint2(acc[0], acc[1]);
        } else {
            o[0] = acc[0];
        }
        if (BL == 0) continue;
        if (cnt) cnt[i] = (uint32_t)C(shift + z[0], shift);
        if (e + 1 == n) break;
        // colex successor: the lowest position that can move up by one
        int t0 = BL - 1;
#pragma unroll
        for (int t = BL - 2; t >= 0; --t)
            if (z[t] + 1 != z[t + 1]) t0 = t;
#pragma unroll
        for (int t = 0; t < BL; ++t)
            if (t <= t0) add_row(z[t]);
#pragma unroll
        for (int t = 0; t < BL; ++t) {
            if (t == t0) z[t] += 1;
            else if (t < t0) z[t] = t;
        }
#pragma unroll
        for (int t = 0; t < BL; ++t)
            if (t <= t0) add_row(z[t]);
    }
}

// the table (index into tab_off) holding flattened entry x
__device__ __forceinline__ int table_of(const BatchCode *cs, uint64_t x) {
    int lo = 0, hi = kBatchTabs - 1;       // last table t with tab_off[t] <= x
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cs->tab_off[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Chunk ch of the table job: entries [ch*tc, ...) of the flattened list
// of the code's tables, one table at a time: the chunk's part of each table
// is split into 64 consecutive runs, one per lane, so that every lane runs
// the same level (a chunk of a short code spans many small tables; lanes
// spread over them would run each level's walk one after another).  The
// wave copies the rows of the set it is in into its own LDS slice (k x dp
// <= kRowsLds words), so that the successor walk's row reads -- a few
// dependent reads per entry -- come from LDS instead of L2.
__device__ void table_chunk(const BatchArgs &A, BatchCode *cs, uint64_t ch, uint32_t tc, uint32_t *lds,
                            LdsU64 *bt) {
    const int lane = threadIdx.x & 63;
    const uint64_t E = uni64(cs->tab_off[kBatchTabs]);
    const int k = (int)uni32((uint32_t)cs->k);
    const uint64_t first = ch * tc;
    const uint64_t end = first + tc < E ? first + tc : E;
    int staged = -1;                     // the set whose rows the LDS slice holds
    for (int t = table_of(cs, first); t < kBatchTabs; ++t) {
        const uint64_t lo = uni64(cs->tab_off[t]), hi = uni64(cs->tab_off[t + 1]);
        if (lo >= end) break;
        const uint64_t x0 = lo > first ? lo : first, x1 = hi < end ? hi : end;
        if (x1 <= x0) continue;          // an empty table
        const int j = t / kTabsPerSet, r0 = t % kTabsPerSet;
        const BatchSet &set = cs->sets[j];
        const int dp = (int)uni32((uint32_t)set.dp), D = (int)uni32((uint32_t)set.D);
        if (j != staged && k * dp <= kRowsLds) {
            const uint32_t *src = (const uint32_t *)uni64((uint64_t)set.rows);
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            for (int w = lane; w < k * dp; w += 64) lds[w] = src[w];
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            staged = j;
        }
        const bool outer = r0 > kBatchMaxB;
        const int b = outer ? r0 - (kBatchMaxB + 1) : r0;
        const int shift = outer ? (int)uni32((uint32_t)set.bcap) : 0;   // outer: rows [0, k-bcap)
        uint32_t *out = (uint32_t *)uni64((uint64_t)(outer ? set.otab[b] : set.rtab[b]));
        uint32_t *cnt = outer ? (uint32_t *)uni64((uint64_t)set.ocnt[b]) : nullptr;
        const int kk = k - shift;
        const uint32_t *rows = staged == j ? lds : (const uint32_t *)uni64((uint64_t)set.rows);
        const uint64_t len = x1 - x0, per = (len + 63) / 64, mine = (uint64_t)lane * per;
        const uint64_t n = mine < len ? (len - mine < per ? len - mine : per) : 0;
        const uint64_t i = x0 - lo + mine;
        if (n > 0) {
            switch (b) {
                case 0: table_run<0>(bt, rows, dp, D, kk, shift, out, cnt, i, n); break;
                case 1: table_run<1>(bt, rows, dp, D, kk, shift, out, cnt, i, n); break;
                case 2: table_run<2>(bt, rows, dp, D, kk, shift, out, cnt, i, n); break;
                case 3: table_run<3>(bt, rows, dp, D, kk, shift, out, cnt, i, n); break;
                case 4: table_run<4>(bt, rows, dp, D, kk, shift, out, cnt, i, n); break;
                case 5: table_run<5>(bt, rows, dp, D, kk, shift, out, cnt, i, n); break;
                default: table_run<6>(bt, rows, dp, D, kk, shift, out, cnt, i, n); break;
            }
        }
    }
}

// What a wave keeps about the job it is working on (read once per job).
struct JobView {
    int c, p, kind;
    BatchJob *jb;
    uint64_t total;
    uint32_t nctr;                // chunk counters of the job
    uint32_t off;                 // the job's arena offset
    // pair jobs
    int j, a, b, b2, k, D, ngroups, gi;
    uint32_t T, offset, L_before;
    uint64_t n_items;
    const uint32_t *rows, *tab, *tab2, *cnt2;
    const GroupEntry *gr;
    const GroupEntry *grl;        // the wave's LDS copy of gr, or nullptr
    uint32_t U;                   // the code's least weight as this wave last saw it (only
                                  // ever above the true one; lowered by the wave's own finds)
};

__device__ __forceinline__ void load_view(const BatchArgs &A, int c, int p, BatchJob *jb, JobView &v) {
    BatchCode *cs = &A.codes[c];
    v.c = c;
    v.p = p;
    v.jb = jb;
    v.kind = (int)uni32((uint32_t)ldc(&jb->kind));
    v.total = uni64(ldc(&jb->total_chunks));
    v.nctr = uni32(ldc(&jb->nctr));
    v.offset = 0;
    v.T = uni32(ldc(&jb->T));      // table job: entries per chunk
    if (v.kind == 0) return;
    v.j = (int)uni32((uint32_t)ldc(&jb->j));
    v.a = (int)uni32((uint32_t)ldc(&jb->a));
    v.b = (int)uni32((uint32_t)ldc(&jb->b));
    v.b2 = (int)uni32((uint32_t)ldc(&jb->b2));
    v.k = (int)uni32((uint32_t)cs->k);
    const BatchSet &set = cs->sets[v.j];
    v.D = (int)uni32((uint32_t)set.D);
    v.rows = (const uint32_t *)uni64((uint64_t)set.rows);
    if (v.b2) {
        v.tab = (const uint32_t *)uni64((uint64_t)set.otab[v.b]);
        v.cnt2 = (const uint32_t *)uni64((uint64_t)set.ocnt[v.b]);
        v.tab2 = (const uint32_t *)uni64((uint64_t)set.rtab[v.b2]);
    } else {
        v.tab = (const uint32_t *)uni64((uint64_t)set.rtab[v.b]);
        v.cnt2 = v.tab2 = nullptr;
    }
    v.n_items = uni64(ldc(&jb->n_items));
    v.offset = uni32(ldc(&jb->offset));
    v.L_before = uni32(ldc(&jb->L_before));
    v.ngroups = (int)uni32(ldc(&jb->ngroups));
    v.gr = job_groups(jb);
    v.grl = nullptr;
    v.gi = 0;
    v.U = uni32(ld_rlx(&cs->U_found));
}

// One chunk of pair job v.p of code v.c.
// Adds the chunk's evaluated combinations to `exec` and lowers `wmin_out`
// to its least weight (without the offset).
template <int D>
__device__ __forceinline__ void pair_chunk(const BatchArgs &A, const uint64_t *lds_binom, JobView &v, uint64_t ch,
                           uint64_t &exec, uint32_t &wmin_out, bool &wrote) {
    BatchCode *cs = &A.codes[v.c];
    BatchJob *jb = v.jb;
    const int lane = threadIdx.x & 63;
    // group of chunk ch: claims from one counter only grow; a move to
    // another counter may go back
    // the job's chunk groups: from the wave's LDS copy (taken when it
    // picked the job up), else by device-scope loads
    auto gbase = [&](int i) {
        return uni64(v.grl ? v.grl[i].chunk_base : ldc(&v.gr[i].chunk_base));
    };
    if (ch < gbase(v.gi)) v.gi = 0;
    while (v.gi + 1 < v.ngroups && gbase(v.gi + 1) <= ch) ++v.gi;
    const GroupEntry *ge = v.gr + v.gi;
    const GroupEntry *gl = v.grl ? v.grl + v.gi : nullptr;
    const uint64_t base = gbase(v.gi), n_rt = uni64(gl ? gl->n_rt : ldc(&ge->n_rt));
    const uint64_t offc = ch - base;
    ChunkGeo g;
    g.lt = uni64(gl ? gl->lt_begin : ldc(&ge->lt_begin)) + offc / n_rt;
    g.i_begin = uni32((uint32_t)(offc % n_rt) * v.T);
    g.i_end = uni32(min(g.i_begin + v.T, uni32(gl ? gl->nr_first : ldc(&ge->nr_first))));
    g.e_first = uni32(gl ? gl->e : ldc(&ge->e));
    g.clip = false;
    // every address and size of the enumeration re-broadcast from lane 0 at
    // the point of use: the table reads stay scalar loads whatever the
    // scheduler loop around this call looks like to the compiler
    const int a = (int)uni32((uint32_t)v.a), b = (int)uni32((uint32_t)v.b);
    // binomials from the block's LDS slice when the subsets are short
    // enough (a dependent chain of global loads per element otherwise)
    const int k_ = (int)uni32((uint32_t)v.k), b2_ = (int)uni32((uint32_t)v.b2);
    const bool lds_b = k_ <= kLdsBinomX && a < kLdsBinomT && b < kLdsBinomT;
    const uint64_t *bt = lds_b ? lds_binom : A.binom;
    const int bs = lds_b ? kLdsBinomT : kBinomT;
    const ItemSrc src{(const uint32_t *)uni64((uint64_t)v.rows), (const uint32_t *)uni64((uint64_t)v.tab),
                      nullptr, bt, bt + a, bt + b, bs, bs,
                      uni64(v.n_items), k_, a, b, b2_,
                      (const uint32_t *)uni64((uint64_t)v.tab2), (const uint32_t *)uni64((uint64_t)v.cnt2), bs};
    constexpr int BI = batch_items(D);
    uint32_t L[BI][D], nr[BI], lmin, ws;
    uint64_t cnt;
    if (v.b2) run_chunk3<D, BI, false>(src, g, L, nr, lmin, cnt, ws);
    else run_chunk<D, BI, false, (D <= kMfmaMaxD) ? kBatchMfmaChains : 0>(src, g, L, nr, lmin, cnt, ws);
    const uint32_t wmin = uni32(wave_min_u32(lmin));
    exec += uni64(wave_sum_u64(cnt));
    if (wmin < wmin_out) wmin_out = wmin;
    if (wmin == kInf) return;
    const uint32_t val = wmin + v.offset;
    if (val >= v.U) return;
    uint32_t old = 0;
    if (lane == 0) old = atomicMin(&cs->U_found, val);
    old = uni32((uint32_t)__shfl((int)old, 0));
    v.U = min(old, val);
    if (old > val) {
        uint32_t hit_i, hit_i2 = 0;
        uint64_t hit_rho;
        const int first =
            v.b2 ? find_witness3<D, BI>(src, g, L, nr, wmin, hit_i, hit_i2, hit_rho)
                 : find_witness<D, BI>(src, g, L, nr, wmin, hit_i, hit_rho);
        if (lane == first) {
            cs->slots[val].pair = (uint32_t)v.p;
            cs->slots[val].i = hit_i;
            cs->slots[val].i2 = hit_i2;
            cs->slots[val].rho = hit_rho;
        }
        wrote = true;
    }
    if (val <= v.L_before && lane == 0) {
        // U reached the bound before this pair: stop handing out its chunks;
        // the pair closes once the chunks already claimed are done
        if (atomicExch(&jb->exit_flag, 1u) == 0u) {
            // chunks handed out so far: counter r hands out at most
            // ceil((total - r) / nctr) of them
            uint64_t claimed = 0;
            for (uint32_t r = 0; r < v.nctr; ++r) {
                const uint64_t t = atomicExch((unsigned long long *)&jb->claim[r].v, 1ull << 62);
                const uint64_t avail = v.total > r ? (v.total - r + v.nctr - 1) / v.nctr : 0;
                claimed += t < avail ? t : avail;
            }
            st_rel(&jb->expected, claimed);
        }
    }
}

// Job p of code c has completed: Algorithm 1's control for that code.  The
// caller's acquire (after the completion count) makes every chunk's
// results visible; the counters are read coherently.
__device__ void advance(const BatchArgs &A, int c, int p, BatchJob *jb) {
    BatchCode *cs = &A.codes[c];
    if ((threadIdx.x & 63) == 0) jb->t_close = wall_clock64();
    const int k = cs->k, n = cs->n, ng = cs->n_gamma;
    const uint32_t singleton = (uint32_t)(n - k + 1);
    if (jb->kind == 0) {           // tables built: first pair, L = 1 (Algorithm 1)
        open_pair(A, c, p + 1, 0, 1, 1u);
        return;
    }
    const int j = jb->j, w = jb->w;
    const uint32_t Uf = uni32(ldc(&cs->U_found));
    const uint64_t executed = uni64(ldc(&jb->executed));
    const bool cut = uni32(ldc(&jb->exit_flag)) && executed < jb->count;
    const uint32_t L = cut ? jb->L_before
                           : (uint32_t)bound_after_dev(k, cs->m_full, cs->k_m, ng, j, w);
    const uint32_t U = min(Uf, singleton);
    if ((threadIdx.x & 63) == 0) {
        jb->L_after = L;
        jb->U_after = U;
    }
    if (cut) { finish_code(A, c, kSlotDone, L, U); return; }
    int j2 = j + 1, w2 = w;
    if (j2 >= ng) { j2 = 0; w2 = w + 1; }
    if (w2 > k || L >= U) { finish_code(A, c, kSlotDone, L, U); return; }
    if (p + 1 >= kBatchMaxPairs || w2 > 64 || binom(A.binom, k, w2) >= (1ull << 63)) {
        finish_code(A, c, -5 /* MINDIST_E_LIMIT */, L, U);
        return;
    }
    open_pair(A, c, p + 1, j2, w2, L);
}

// Next chunk of job jb (total chunks, nctr counters) for this wave, or ~0
// once every counter is drained.  ctr: the counter tried next; dmask: the
// counters known drained -- found by this wave, or by others (the job's
// shared mask, returned by the one atomic a wave spends on a drained
// counter), so that at the end of a job each wave makes about two claims
// instead of one per counter.
__device__ __forceinline__ uint64_t claim_chunk(BatchJob *jb, uint64_t total, uint32_t nctr, uint32_t &ctr,
                                uint32_t &dmask) {
    const uint32_t all = (1u << nctr) - 1u;
    while ((dmask & all) != all) {
        const uint32_t r = ctr;
        const uint64_t t = wave_fetch_add(&jb->claim[r].v, 1ull);
        if (t < total) {
            const uint64_t ch = (uint64_t)r + t * nctr;
            if (ch < total) return ch;
        }
        uint32_t seen = 0;
        if ((threadIdx.x & 63) == 0) seen = atomicOr(&jb->drained_mask, 1u << r);
        dmask |= uni32((uint32_t)__shfl((int)seen, 0)) | (1u << r);
        for (uint32_t q = 1; q <= nctr; ++q) {
            const uint32_t r2 = (r + q) % nctr;
            if (!(dmask & (1u << r2))) { ctr = r2; break; }
        }
    }
    return ~0ull;
}

// Add a wave's `done` completed chunks of job p of code c (with their
// `exec` evaluated combinations and least weight `wmin` + offset) to the
// job; the flush that brings the job's count to `expected` closes the job
// and applies Algorithm 1's control.  The counts travel in device-scope
// atomics; only a wave that wrote plain data since its last flush (table
// entries, a witness slot) releases it first -- a release at device scope
// writes back the XCD's whole L2.
__device__ __noinline__ void flush(const BatchArgs &A, int c, int p, BatchJob *jb, uint64_t done, uint64_t exec,
                      uint32_t wmin, uint32_t offset, bool wrote) {
    if (done == 0) return;
    const int lane = threadIdx.x & 63;
    uint64_t prev = 0, expected = 0;
    if (lane == 0) {
        if (exec) atomicAdd((unsigned long long *)&jb->executed, (unsigned long long)exec);
        if (wmin != kInf) atomicMin(&jb->pair_min, wmin + offset);
    }
    // the count atomics (performed at device scope) complete before `done`
    // is added: a release at workgroup scope waits for them without cache
    // maintenance; plain data written since the last flush needs the
    // device-scope release
    if (wrote) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane == 0) {
        prev = __hip_atomic_fetch_add((unsigned long long *)&jb->done, (unsigned long long)done,
                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        expected = __hip_atomic_fetch_add((unsigned long long *)&jb->expected, 0ull, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    }
    prev = uni64((uint64_t)__shfl((long long)prev, 0));
    expected = uni64((uint64_t)__shfl((long long)expected, 0));
    if (prev + done == expected) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        advance(A, c, p, jb);
    }
}

// Serving: copy the codes the host admitted while this launch runs to the
// device.  The host writes a code's descriptor and packed rows into its
// slot's inbox entry (pinned host memory), the slot into the ring, then the
// count; the wave holding the admission lock copies each entry (rows into
// the code's pool range, the descriptor from its second line on), clears
// the first line's state and turns the slot PENDING after a release, so a
// wave that sees the status reads the rest from memory.  A slot and a pool
// range are used at most once per launch: no wave can still hold anything
// of what they held before, and no XCD's L2 a stale copy of them.
__device__ __noinline__ void admit_codes(const BatchArgs &A) {
    const int lane = threadIdx.x & 63;
    uint32_t got = 0;
    if (lane == 0) got = atomicCAS(&A.g->admit_lock, 0u, 1u) == 0u ? 1u : 0u;
    if (!uni32((uint32_t)__shfl((int)got, 0))) return;
    // the entries were written before the count
    const uint32_t pub = uni32(__hip_atomic_load(A.admit_count, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM));
    uint32_t done = uni32(ld_rlx(&A.g->admit_done));
    constexpr int kLine0 = 128 / 16;
    for (; done < pub; ++done) {
        const uint32_t s = uni32(__hip_atomic_load(A.admit_ring + done % (uint32_t)A.n_codes,
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM));
        if (s >= (uint32_t)A.n_codes) continue;          // never written so by the host
        const ServeInbox *in = A.inbox + s;
        BatchCode *cs = A.codes + s;
        const uint4 *src = reinterpret_cast<const uint4 *>(&in->code);
        uint4 *dst = reinterpret_cast<uint4 *>(cs);
        for (int q = kLine0 + lane; q < (int)(sizeof(BatchCode) / 16); q += 64) dst[q] = src[q];
        uint4 *rd = reinterpret_cast<uint4 *>(uni64(in->rows_dst));
        const uint32_t rq = min(uni32(in->rows_bytes), (uint32_t)kInboxRowsBytes) / 16;
        const uint4 *rs = reinterpret_cast<const uint4 *>(in->rows);
        for (uint32_t q = lane; q < rq; q += 64) rd[q] = rs[q];
        if (lane == 0) {
            __hip_atomic_store(&cs->njobs, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&cs->drained, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&cs->U_found, kInf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        // every lane's stores complete, lane 0's release writes them back
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {
            atomicAdd(&A.g->live0, 1u);
            st_rel(&cs->status, (int32_t)kSlotPending);
        }
    }
    if (lane == 0) {
        __hip_atomic_store(&A.g->admit_done, pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(A.admit_ack, pub, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&A.g->admit_lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// A wave that found nothing to do sleeps before it looks again, twice as
// long after each empty look, from ~0.85 us up to ~54 us (s_sleep 32 is
// 2048 clocks).  Thousands of idle waves re-reading the few lines of the
// code descriptors every ~0.1 us had queued the working waves' own memory
// accesses behind them: a chunk of a short pair of a code running alone
// took ~37 us, ~14 us with the back-off; an eligible picker among hundreds
// still wakes within a fraction of a microsecond.
__device__ __forceinline__ void idle_backoff(uint32_t &idle) {
    const uint32_t n = 1u << (idle < 6u ? idle : 6u);
    for (uint32_t q = 0; q < n; ++q) __builtin_amdgcn_s_sleep(32);
    if (idle < 6u) ++idle;
}

}  // namespace

// At most 256 VGPRs (2 waves per SIMD, 2 blocks of 256 per CU): the
// matrix-core operands and products of pairs of up to 4 words take about
// 200 of them; at 128 the enumeration loops themselves would spill.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void persistent_batch_kernel(BatchArgs A) {
    // one slice per wave for the rows of the set whose tables it builds
    __shared__ uint32_t s_rows[4 * kRowsLds];
    uint32_t *const my_rows = s_rows + (threadIdx.x >> 6) * kRowsLds;
    __shared__ uint64_t s_binom[kLdsBinomX * kLdsBinomT];
    for (int q = threadIdx.x; q < kLdsBinomX * kLdsBinomT; q += blockDim.x)
        s_binom[q] = binom(A.binom, q / kLdsBinomT, q % kLdsBinomT);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const uint32_t wave = uni32(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    const int nc = A.n_codes;
    int cur = (int)(wave % (uint32_t)nc);
    const uint64_t t_start = wall_clock64();
    JobView v;
    bool have = false;             // v describes a job this wave claims on
    // arena offset of the last job this wave found drained (an integer: a
    // loop-carried pointer here costs the enumeration its scalar loads)
    uint32_t drained = 0xFFFFFFFFu;
    // claiming state and this wave's completed chunks of v's job not yet
    // added to it
    uint32_t ctr = 0, dmask = 0, pmin = kInf, visit = 0;
    uint64_t pdone = 0, pexec = 0;
    bool wrote = false;            // plain stores since the last flush (tables, a witness slot)
    uint32_t idle = 0;             // empty looks since this wave last took up a job
    // profile: ticks in table chunks, enumeration chunks and flushes
    uint64_t tk_table = 0, tk_pair = 0, tk_flush = 0, n_table = 0, n_pair = 0;
    for (;;) {
        bool stop = A.deadline_ticks && wall_clock64() - t_start > A.deadline_ticks;
        if (A.serving) {
            // wave 0 watches the host's flag (pinned memory, read over the
            // bus) and mirrors it on the device for every other wave
            if (wave == 0) {
                const uint32_t hs = A.host_stop ? __hip_atomic_load(A.host_stop, __ATOMIC_RELAXED,
                                                                    __HIP_MEMORY_SCOPE_SYSTEM)
                                                : 1u;
                if (uni32(hs) != 0 && lane == 0)
                    __hip_atomic_store(&A.g->stop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            stop = stop || uni32(ld_rlx(&A.g->stop)) != 0;
        } else if (uni32(ld_rlx(&A.g->codes_done)) >= (uint32_t)nc) {
            stop = true;
        }
        if (!stop && A.admit_count && (wave & 63) == 0) {
            // one wave in 64 watches for codes admitted while the launch runs
            const uint32_t pub = uni32(__hip_atomic_load(A.admit_count, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_SYSTEM));
            if (pub != uni32(ld_rlx(&A.g->admit_done))) admit_codes(A);
        }
        if (stop) {
            // every chunk this wave claimed is complete: count it before leaving
            if (have) flush(A, v.c, v.p, v.jb, pdone, pexec, pmin, v.offset, wrote);
            if (lane == 0) {
                atomicAdd((unsigned long long *)&A.g->ticks_table, (unsigned long long)tk_table);
                atomicAdd((unsigned long long *)&A.g->ticks_pair, (unsigned long long)tk_pair);
                atomicAdd((unsigned long long *)&A.g->ticks_flush, (unsigned long long)tk_flush);
                atomicAdd((unsigned long long *)&A.g->chunks_table, (unsigned long long)n_table);
                atomicAdd((unsigned long long *)&A.g->chunks_pair, (unsigned long long)n_pair);
            }
            break;
        }
        if (have) {
            // the visit quantum spreads waves over short codes' jobs; a job
            // of 1024 chunks or more keeps its waves (leaving it every few
            // chunks only added flushes and pick-ups: heavy stratum 24.1 ->
            // 22.9 s)
            const bool turn_over = A.quantum && visit >= A.quantum && v.total < kQuantumJobChunks;
            const uint64_t ch = turn_over ? ~0ull : claim_chunk(v.jb, v.total, v.nctr, ctr, dmask);
            if (ch != ~0ull) {
                const uint64_t t0 = wall_clock64();
                if (v.kind == 0) {
                    table_chunk(A, &A.codes[v.c], ch, v.T, my_rows, (LdsU64 *)s_binom);
                    wrote = true;
                    tk_table += wall_clock64() - t0;
                    n_table += 1;
                } else {
                    switch (v.D) {
                        case 1: pair_chunk<1>(A, s_binom, v, ch, pexec, pmin, wrote); break;
                        case 2: pair_chunk<2>(A, s_binom, v, ch, pexec, pmin, wrote); break;
                        case 3: pair_chunk<3>(A, s_binom, v, ch, pexec, pmin, wrote); break;
                        case 4: pair_chunk<4>(A, s_binom, v, ch, pexec, pmin, wrote); break;
                        case 5: pair_chunk<5>(A, s_binom, v, ch, pexec, pmin, wrote); break;
                        case 6: pair_chunk<6>(A, s_binom, v, ch, pexec, pmin, wrote); break;
                        case 7: pair_chunk<7>(A, s_binom, v, ch, pexec, pmin, wrote); break;
                        default: pair_chunk<8>(A, s_binom, v, ch, pexec, pmin, wrote); break;
                    }
                    tk_pair += wall_clock64() - t0;
                    n_pair += 1;
                }
                pdone += 1;
                visit += 1;
                continue;
            }
            // this job is drained for this wave (tell the others), or this
            // visit's share is used up: count its chunks and move on
            if (!turn_over && lane == 0) atomicMax(&A.codes[v.c].drained, v.p + 1);
            const uint64_t t0 = wall_clock64();
            flush(A, v.c, v.p, v.jb, pdone, pexec, pmin, v.offset, wrote);
            wrote = false;
            tk_flush += wall_clock64() - t0;
            if (!turn_over) drained = v.off;
            have = false;
            cur = turn_over ? (v.c + 1) % nc : v.c;
        }
        // find a code with work: 64 slots per look, relaxed reads of the
        // status, the jobs opened and the drained hint (a code whose open
        // job is fully claimed is passed over without touching the job)
        const int probe = (cur + lane) % nc;
        const int32_t s = (int32_t)__hip_atomic_load(&A.codes[probe].status, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
        const int32_t pj = __hip_atomic_load(&A.codes[probe].njobs, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        const int32_t pd = __hip_atomic_load(&A.codes[probe].drained, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long live =
            __ballot(s == kSlotPending || (s == kSlotActive && pj > 0 && pd < pj));
        if (!live) {
            cur = (cur + 64) % nc;
            idle_backoff(idle);
            continue;
        }
        const int pick = __builtin_ctzll(live);
        const int c = (cur + pick) % nc;
        const int32_t st = (int32_t)uni32((uint32_t)__shfl(s, pick));
        BatchCode *cs = &A.codes[c];
        if (st == kSlotPending) {
            // first wave to see the slot opens its table job
            int32_t won = 0;
            if (lane == 0)
                won = atomicCAS(&cs->status, (int32_t)kSlotPending, (int32_t)kSlotOpening) == kSlotPending;
            if (uni32((uint32_t)__shfl(won, 0))) open_tables(A, c);
            continue;
        }
        const int nj = (int)uni32((uint32_t)__hip_atomic_load(&cs->njobs, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT));
        if (nj <= 0) { cur = (c + 1) % nc; continue; }
        const int p = nj - 1;
        // a relaxed look first (no fence while waiting on a drained job)
        const uint32_t off0 = uni32(__hip_atomic_load(&cs->job[p], __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT));
        if (off0 == drained) {     // still waiting for its last chunks
            cur = (c + 1) % nc;
            idle_backoff(idle);
            continue;
        }
        // no acquire fence: the job's record and groups are read with
        // device-scope loads (ldc) through the published offset, and its
        // tables were released by the waves that built them (their flushes)
        // before the pair that reads them was opened
        const uint32_t off = off0;
        BatchJob *jb = job_at(A, off);
        {
            // A job of few chunks is left to a subset of the waves (rotated
            // by code): every wave that looks at a job claims from it and
            // marks it drained with device-scope atomics on a few lines, so
            // thousands of idle waves falling on a one-chunk pair had cost
            // each pair of a code running alone ~0.35 ms.  With at most 4
            // live codes, one picker per chunk (at least 64): the waves
            // that would only find the job drained add claims and
            // completion atomics to its lines (a code alone: 10-15 % per
            // pair); with more, 4 per chunk (at least 256) spread the waves
            // better over many short jobs
            const uint64_t total = uni64(ldc(&jb->total_chunks));
            const uint32_t waves = gridDim.x * (blockDim.x >> 6);
            const uint32_t l0 = uni32(ld_rlx(&A.g->live0)), cd = uni32(ld_rlx(&A.g->codes_done));
            const bool few = (l0 ? l0 : (uint32_t)nc) <= cd + kFewLiveCodes;
            const uint64_t per = few ? kPickersPerChunkFew : kPickersPerChunk;
            const uint64_t lo = few ? kPickersMinFew : kPickersMin;
            const uint64_t want = total * per > lo ? total * per : lo;
            if (want < waves) {
                const uint32_t rank = (wave + (uint32_t)c * 0x9E3779B1u % waves) % waves;
                if (rank >= want) {
                    drained = off;
                    cur = (c + 1) % nc;
                    continue;
                }
            }
        }
        load_view(A, c, p, jb, v);
        if (v.kind == 1 && (uint32_t)v.ngroups * sizeof(GroupEntry) <= kRowsLds * sizeof(uint32_t)) {
            // the groups into this wave's LDS slice (one round of parallel
            // device-scope loads instead of a dependent chain per chunk)
            const uint64_t *src = reinterpret_cast<const uint64_t *>(v.gr);
            uint64_t *dst = reinterpret_cast<uint64_t *>(my_rows);
            const int words = v.ngroups * (int)(sizeof(GroupEntry) / sizeof(uint64_t));
            __builtin_amdgcn_wave_barrier();
            for (int q = lane; q < words; q += 64) dst[q] = ldc(src + q);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            v.grl = reinterpret_cast<const GroupEntry *>(my_rows);
        }
        v.off = off;
        ctr = wave % v.nctr;
        dmask = 0;
        pdone = pexec = 0;
        pmin = kInf;
        visit = 0;
        have = true;
        idle = 0;
        cur = c;
    }
}

int persistent_resident_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, persistent_batch_kernel, 256, 0) != hipSuccess)
        return 0;
    return n;
}

// eight threads per 128-byte line, 16 bytes each
__global__ __launch_bounds__(256) void gather_lines_kernel(const unsigned char *arena, const uint32_t *src,
                                                           uint32_t n, unsigned char *dst) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t line = t >> 3, part = t & 7;
    if (line >= n) return;
    const uint4 *from = reinterpret_cast<const uint4 *>(arena + (size_t)src[line] * 128) + part;
    uint4 *to = reinterpret_cast<uint4 *>(dst + line * 128) + part;
    *to = *from;
}

int launch_gather_lines(const unsigned char *arena, const uint32_t *src, uint32_t n, unsigned char *dst,
                        void *stream) {
    if (n == 0) return 0;
    const uint64_t threads = (uint64_t)n * 8;
    hipLaunchKernelGGL(gather_lines_kernel, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, arena, src, n, dst);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_persistent(const BatchArgs &a, int blocks, void *stream) {
    hipLaunchKernelGGL(persistent_batch_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace md
