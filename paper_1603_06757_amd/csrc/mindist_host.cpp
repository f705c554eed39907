// mindist_host.cpp -- the single-code path: context creation (information
// sets and Gamma_j from mindist_plan), the pair loop of Algorithm 1 with
// one enumeration launch per pair, witness reconstruction, and the C ABI of
// the single-code entry points.  L is raised after every Gamma_j by default,
// or by the printed per-level update when MINDIST_OPT_TERM = 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <tuple>
#include <string>
#include <vector>

#include "../../include/mindist.h"
#include "mindist_internal.h"
#include "mindist_plan.h"
#include "mindist_pool.h"
#include "mindist_walk.h"

using namespace md;

namespace md {
const char *last_error_text();
}

#define HIPCHK(expr)                                                                  \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(MINDIST_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

extern "C" const char *mindist_last_error(void) { return md::last_error_text(); }

static PairView view_of(const mindist_pair &r) {
    return PairView{r.j, r.w, r.L_before, r.L_after, r.U_after, r.pair_min, r.count, r.executed};
}

namespace {

struct GammaDev {
    int D = 0, DP = 0;         // dwords carried / stored per row
    bool stripped = false;     // identity columns removed (weight offset w)
    uint32_t *rows = nullptr;  // device, k x DP
    uint32_t *h_rows = nullptr;   // pinned staging of rows (source of the upload)
    // saved-sum tables keyed by (kind, size, shift): kind 0 left, 1 right
    // (shift 0) or outer (shift = b2, with inner counts)
    std::map<std::tuple<int, int, int>, std::pair<uint32_t *, uint32_t *>> tabs;
    int bcap = 0;              // largest b whose table fits the cap
};

struct PairPlan {
    int a = 0, b = 0, b2 = 0;   // |X| per lane, outer |Y1| (or right |Y|), inner |Y2|
    uint32_t T = 0;
    uint32_t n_rt = 0;         // right tiles (right-major order)
    uint64_t n_items = 0, total_chunks = 0;
    int ngroups = 0;
};

}  // namespace

// ---------------------------------------------------------------------------
struct mindist_ctx {
    Plan P;
    int n_gamma = 0;           // enumerated sets (partial included unless dropped)
    std::vector<GammaDev> gd;
    // options
    int term_per_level = 0, midpair_exit = 1, partial_policy = kPartialAlways, verify = 0, profile = 0;
    int64_t deadline_ms = 0;
    uint64_t cancel_after = 0;
    uint32_t tile_t = 0;       // 0: chosen per pair
    int blocks_per_cu = 0;     // 0: blocks_per_cu_for's default
    int items = 4;             // lane items per chunk (kernel template B)
    int order = 0;             // chunk order: 0 left-tile-major, 1 right-tile-major
    int counters = kCounters;  // chunk dispensers (1 or kCounters)
    int left_tables = 1;       // read left subsets from saved tables when they fit
    int mfma = 1;              // full right blocks of D <= 4 pairs on the int8 matrix cores
    uint64_t table_cap = kTableCapDefault;
    uint64_t min_items = 0;    // left subsets a pair's split should give (0 = balanced split)
    uint32_t inject_u = 0;             // testing: initial least weight on the device (0 = off)
    uint64_t speculate = 1ull << 28;   // launch the next pair before the current one's result
                                       // is read when it has at most this many combinations
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0, cus = 256;
    double wall_hz = 1e8;      // device wall-clock rate
    // device buffers
    const uint64_t *d_binom = nullptr;   // shared per device
    DevState *d_state = nullptr;
    int max_pairs = 0;
    int groups_cap = 0;                 // chunk groups of one pair at most (k + 2)
    uint64_t *d_rprefix = nullptr, *h_rprefix = nullptr;
    size_t rprefix_cap = 0;
    // pinned host staging
    PairMail *h_mail = nullptr, *d_mail = nullptr;   // pinned mailboxes: pair p uses p % kMailRing
    WavePart *d_parts = nullptr;        // per-wave totals of the running pair
    uint64_t parts_cap = 0;
    // plans of the pairs met so far, by (j, w) and the kernel shape options,
    // with the device copy of their chunk groups
    std::map<std::array<uint64_t, 6>, std::pair<PairPlan, const GroupEntry *>> plan_cache;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<hipEvent_t> pair_ev;    // profile: start/end event of every pair
    std::vector<uint64_t> rprefix_host;
    // last run
    std::vector<mindist_pair> trace;
    bool have_run = false;
    // no-allocation mode (mindist_run_noalloc): every device buffer lies in
    // a fixed region the caller provides; the mailboxes are device memory
    // read back by copies; each pair's tables are rebuilt in one arena
    int noalloc = 0;
    unsigned char *arena = nullptr;
    uint64_t arena_bytes = 0, arena_used = 0;
    GroupEntry *d_groups_fixed = nullptr;   // the current pair's chunk groups
    std::vector<PairMail> mail_host;        // h_mail's storage in this mode
};

static void free_ctx(mindist_ctx *c) {
    if (!c) return;
    if (c->noalloc) { delete c; return; }   // nothing of its own on the device
    // a launched-ahead pair may still read this context's buffers
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (auto &g : c->gd) {
        dev_free(g.rows);
        pinned_free(g.h_rows);
        for (auto &kv : g.tabs) {
            dev_free(kv.second.first);
            dev_free(kv.second.second);
        }
    }
    dev_free(c->d_state);
    dev_free(c->d_rprefix);
    pinned_free(c->h_rprefix);
    mapped_free(c->h_mail);
    dev_free(c->d_parts);
    event_put(c->ev0);
    event_put(c->ev1);
    for (hipEvent_t e : c->pair_ev) event_put(e);
    if (c->own_stream && c->stream) stream_put(c->stream);
    delete c;
}

static int upload_gamma(mindist_ctx *c, int j) {
    const Plan &P = c->P;
    GammaDev &g = c->gd[j];
    const std::vector<int> cols = carried_columns(P, j);
    const bool full = j < P.m_full;
    g.stripped = full;
    g.D = (int)((cols.size() + 31) / 32);
    g.DP = dp_of_host(g.D);
    // packed rows staged in pinned memory the context keeps, so the copy is
    // asynchronous and creation never waits for it (kernels that read the
    // rows follow it in stream order)
    const size_t words = (size_t)P.k * g.DP;
    g.h_rows = static_cast<uint32_t *>(pinned_alloc(words * 4));
    g.rows = static_cast<uint32_t *>(dev_alloc(words * 4));
    if (!g.rows || !g.h_rows) return fail(MINDIST_E_NOMEM, "allocation of Gamma rows failed");
    std::memset(g.h_rows, 0, words * 4);
    for (int r = 0; r < P.k; ++r) pack_row(&P.gamma[j][(size_t)r * P.W], cols, &g.h_rows[(size_t)r * g.DP], g.DP);
    HIPCHK(hipMemcpyAsync(g.rows, g.h_rows, words * 4, hipMemcpyHostToDevice, c->stream));
    const Binom &B = BN();
    g.bcap = 0;
    for (int b = 1; b <= 16 && b <= P.k; ++b) {
        uint64_t ent = B(P.k, b);
        if (ent >= (1ull << 31) || ent * (uint64_t)g.DP * 4 > c->table_cap) break;
        g.bcap = b;
    }
    return MINDIST_OK;
}

// saved sums of r-subsets of the rows of Gamma_j (see TableArgs): built once
// per (kind, r, shift) and kept with the context.  kind 0 = left table,
// 1 = right table (shift 0) or outer table of a three-level split (shift b2).
static int get_table(mindist_ctx *c, int j, int r, int kind, int shift, uint32_t **out,
                     uint32_t **cnt_out = nullptr) {
    GammaDev &g = c->gd[j];
    const auto key = std::make_tuple(kind, r, shift);
    auto it = g.tabs.find(key);
    if (it != g.tabs.end()) {
        *out = it->second.first;
        if (cnt_out) *cnt_out = it->second.second;
        return MINDIST_OK;
    }
    // a plain table of level r >= 2 is extended from level r - 1 (built
    // first if missing): one row per entry instead of r
    uint32_t *prev = nullptr;
    if (shift == 0 && r >= 2) {
        int e = get_table(c, j, r - 1, kind, 0, &prev);
        if (e) return e;
    }
    const uint64_t ent = BN()(c->P.k - shift, r);
    uint32_t *t = nullptr, *cn = nullptr;
    if (c->noalloc) {
        // the arena of the fixed region (reset before every pair)
        auto take = [&](uint64_t bytes) -> uint32_t * {
            const uint64_t at = (c->arena_used + 255) & ~255ull;
            if (at + bytes > c->arena_bytes) return nullptr;
            c->arena_used = at + bytes;
            return reinterpret_cast<uint32_t *>(c->arena + at);
        };
        t = take(ent * g.DP * 4);
        cn = shift ? take(ent * 4) : nullptr;
        if (!t || (shift && !cn))
            return fail(MINDIST_E_LIMIT, "saved-sum tables exceed the fixed region");
    } else {
        t = static_cast<uint32_t *>(dev_alloc(ent * g.DP * 4));
        cn = shift ? static_cast<uint32_t *>(dev_alloc(ent * 4)) : nullptr;
        if (!t || (shift && !cn)) {
            dev_free(t);
            dev_free(cn);
            return fail(MINDIST_E_NOMEM, "saved-sum table allocation failed");
        }
    }
    TableArgs ta{g.rows, c->d_binom, t, cn, ent, c->P.k, r, g.DP, kind ? 1 : 0, shift, prev};
    if (launch_build_table(ta, g.D, c->stream)) {
        if (!c->noalloc) {
            dev_free(t);
            dev_free(cn);
        }
        return fail(MINDIST_E_HIP, "table kernel launch failed");
    }
    g.tabs[key] = {t, cn};
    *out = t;
    if (cnt_out) *cnt_out = cn;
    return MINDIST_OK;
}

// a left table is used when it fits the same cap as the right tables
static bool left_table_fits(const mindist_ctx *c, int j, int a) {
    const uint64_t ent = BN()(c->P.k, a);
    return ent < (1ull << 31) && ent * (uint64_t)c->gd[j].DP * 4 <= c->table_cap;
}

extern "C" int mindist_plan(const uint64_t *G, int n, int k, int *sets, int *m_full,
                            int *k_partial, uint64_t *gammas) {
    Plan P;
    int e = make_plan(G, n, k, P);
    if (e) return e;
    if (m_full) *m_full = P.m_full;
    if (k_partial) *k_partial = P.k_m;
    if (sets) {
        int o = 0;
        for (auto &s : P.sets) for (int c : s) sets[o++] = c;
    }
    if (gammas)
        for (size_t j = 0; j < P.gamma.size(); ++j)
            std::memcpy(gammas + j * (size_t)P.k * P.W, P.gamma[j].data(),
                        sizeof(uint64_t) * P.k * P.W);
    return MINDIST_OK;
}

extern "C" int mindist_bound_after(int k, int m_full, int k_partial, int include_partial,
                                   int j, int w) {
    const int ng = m_full + ((include_partial && k_partial >= 1) ? 1 : 0);
    if (k < 1 || m_full < 0 || j < 0 || j >= ng || w < 1) return fail(MINDIST_E_ARG, "bad bound query");
    return bound_after(k, m_full, k_partial, ng, j, w);
}

extern "C" int mindist_schedule(int k, int m_full, int k_partial, int partial_policy, int per_level,
                                int32_t *out, int cap, int *n_out) {
    if (k < 1 || m_full < 1 || k_partial < 0 || k_partial >= k || partial_policy < 0 ||
        partial_policy > 2 || cap < 0 || (cap > 0 && !out) || !n_out)
        return fail(MINDIST_E_ARG, "schedule: bad arguments");
    const Schedule S(k, m_full, k_partial, partial_policy);
    PairPos p = S.first();
    int t = 0, L = 1;
    for (bool more = true; more; more = S.next(p, &p), ++t) {
        L = S.L_after(p, per_level != 0, L);
        if (t < cap) {
            out[4 * t] = p.j;
            out[4 * t + 1] = p.h;
            out[4 * t + 2] = p.g;
            out[4 * t + 3] = L;
        }
    }
    *n_out = t;
    return MINDIST_OK;
}

extern "C" int mindist_certify(const mindist_cert_spec *spec, const mindist_pair *pairs, int n_pairs,
                               int d, int L_final, int exited_midpair) {
    if (!spec || (n_pairs > 0 && !pairs) || n_pairs < 0) return fail(MINDIST_E_ARG, "certify: bad arguments");
    if (spec->k < 1 || spec->n <= spec->k || spec->m_full < 1 || spec->k_partial < 0 ||
        spec->k_partial >= spec->k || spec->partial_policy < 0 || spec->partial_policy > 2)
        return fail(MINDIST_E_ARG, "certify: bad spec");
    CertSpec cs;
    cs.n = spec->n;
    cs.k = spec->k;
    cs.sched = Schedule(spec->k, spec->m_full, spec->k_partial, spec->partial_policy);
    cs.per_level = spec->per_level != 0;
    cs.midpair_exit = spec->midpair_exit != 0;
    std::vector<PairView> v((size_t)n_pairs);
    for (int t = 0; t < n_pairs; ++t) v[t] = view_of(pairs[t]);
    return certify_trace(cs, v.data(), n_pairs, d, L_final, exited_midpair);
}

extern "C" int mindist_colex_unrank(uint64_t rank, int r, int hi, int *out) {
    if (!out || r < 0 || r > 64 || hi < r || hi > 512) return fail(MINDIST_E_ARG, "bad unrank query");
    if (rank >= BN()(hi, r)) return fail(MINDIST_E_ARG, "rank out of range");
    colex_unrank(rank, r, hi, out);
    return MINDIST_OK;
}

extern "C" int mindist_create(const uint64_t *G, int n, int k, mindist_ctx **out) {
    if (!out) return fail(MINDIST_E_ARG, "out is NULL");
    *out = nullptr;
    mindist_ctx *c = new (std::nothrow) mindist_ctx();
    if (!c) return fail(MINDIST_E_NOMEM, "context allocation failed");
    int e = make_plan(G, n, k, c->P);
    if (e) { free_ctx(c); return e; }
    c->n_gamma = (int)c->P.sets.size();
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        free_ctx(c);
        return fail(MINDIST_E_HIP, "no HIP device");
    }
    hipDeviceProp_t prop;
#define CHK(expr) do { hipError_t e_ = (expr); if (e_ != hipSuccess) { free_ctx(c); \
        return fail(MINDIST_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); } } while (0)
    CHK(hipGetDevice(&c->device));
    CHK(hipGetDeviceProperties(&prop, c->device));
    c->cus = prop.multiProcessorCount;
    {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) == hipSuccess && khz > 0)
            c->wall_hz = khz * 1000.0;
    }
#undef CHK
    c->stream = stream_get();
    c->own_stream = true;
    c->d_binom = device_binom_from(BN().t.data());
    c->max_pairs = c->n_gamma * std::min(k, MINDIST_MAX_LEVEL) + 1;
    c->d_state = static_cast<DevState *>(dev_alloc(state_bytes(c->max_pairs)));
    c->groups_cap = k + 2;
    {
        void *dm = nullptr;
        c->h_mail = static_cast<PairMail *>(mapped_alloc(kMailRing * sizeof(PairMail), &dm));
        c->d_mail = static_cast<PairMail *>(dm);
    }
    c->ev0 = event_get();
    c->ev1 = event_get();
    if (!c->stream || !c->d_binom || !c->d_state || !c->h_mail || !c->ev0 || !c->ev1) {
        free_ctx(c);
        return fail(MINDIST_E_NOMEM, "device or pinned allocation failed");
    }
    c->gd.resize(c->n_gamma);
    for (int j = 0; j < c->n_gamma; ++j) {
        e = upload_gamma(c, j);
        if (e) { std::string m = md::last_error_text(); free_ctx(c); return fail(e, m); }
    }
    *out = c;
    return MINDIST_OK;
}

extern "C" void mindist_destroy(mindist_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
}

extern "C" int mindist_set_option(mindist_ctx *c, int key, int64_t v) {
    if (!c) return fail(MINDIST_E_ARG, "ctx is NULL");
    c->plan_cache.clear();        // shape options and the table cap change the plans
    switch (key) {
        case MINDIST_OPT_TERM: c->term_per_level = v ? 1 : 0; break;
        case MINDIST_OPT_MIDPAIR_EXIT: c->midpair_exit = v ? 1 : 0; break;
        case MINDIST_OPT_PARTIAL:
            if (v < 0 || v > 2) return fail(MINDIST_E_ARG, "partial policy must be 0, 1 or 2");
            c->partial_policy = (int)v; break;
        case MINDIST_OPT_VERIFY: c->verify = v ? 1 : 0; break;
        case MINDIST_OPT_STREAM:
            if (c->stream) (void)hipStreamSynchronize(c->stream);
            if (c->own_stream && c->stream) stream_put(c->stream);
            if (v) { c->stream = (hipStream_t)v; c->own_stream = false; }
            else {
                c->stream = stream_get();
                c->own_stream = true;
                if (!c->stream) return fail(MINDIST_E_HIP, "stream creation failed");
            }
            break;
        case MINDIST_OPT_DEADLINE_MS: c->deadline_ms = v < 0 ? 0 : v; break;
        case MINDIST_OPT_TILE_T:
            if (v < 0 || v > (1 << 20)) return fail(MINDIST_E_ARG, "tile_t out of range");
            c->tile_t = (uint32_t)v; break;
        case MINDIST_OPT_LEFT_TABLES: c->left_tables = v ? 1 : 0; break;
        case MINDIST_OPT_MFMA: c->mfma = v ? 1 : 0; break;
        case MINDIST_OPT_CHUNK_ORDER: c->order = v ? 1 : 0; break;
        case MINDIST_OPT_SPECULATE:
            if (v < 0) return fail(MINDIST_E_ARG, "speculate must be >= 0");
            c->speculate = (uint64_t)v; break;
        case MINDIST_OPT_INJECT_U:
            if (v < 0 || v > c->P.n) return fail(MINDIST_E_ARG, "inject_u must be in 0..n");
            c->inject_u = (uint32_t)v; break;
        case MINDIST_OPT_MIN_ITEMS:
            if (v < 0 || v > (int64_t)1 << 40) return fail(MINDIST_E_ARG, "min_items out of range");
            c->min_items = (uint64_t)v; break;
        case MINDIST_OPT_COUNTERS:
            if (v != 1 && v != kCounters) return fail(MINDIST_E_ARG, "counters must be 1 or 8");
            c->counters = (int)v; break;
        case MINDIST_OPT_BLOCKS_PER_CU:
            if (v < 0 || v > 64) return fail(MINDIST_E_ARG, "blocks_per_cu out of range");
            c->blocks_per_cu = (int)v; break;
        case MINDIST_OPT_PROFILE: c->profile = v ? 1 : 0; break;
        case MINDIST_OPT_LANE_ITEMS:
            if (v != 2 && v != 4) return fail(MINDIST_E_ARG, "lane items must be 2 or 4");
            c->items = (int)v; break;
        case MINDIST_OPT_CANCEL_AFTER_CHUNKS: c->cancel_after = v < 0 ? 0 : (uint64_t)v; break;
        case MINDIST_OPT_TABLE_MIB: {
            if (v < 1 || v > (1 << 16)) return fail(MINDIST_E_ARG, "table cap out of range");
            c->table_cap = (uint64_t)v << 20;
            const Binom &B = BN();
            for (auto &g : c->gd) {
                g.bcap = 0;
                for (int b = 1; b <= 16 && b <= c->P.k; ++b) {
                    uint64_t ent = B(c->P.k, b);
                    if (ent >= (1ull << 31) || ent * (uint64_t)g.DP * 4 > c->table_cap) break;
                    g.bcap = b;
                }
            }
            break;
        }
        default: return fail(MINDIST_E_ARG, "unknown option " + std::to_string(key));
    }
    return MINDIST_OK;
}

extern "C" int mindist_info(const mindist_ctx *c, int *m_full, int *k_partial, int *n_gamma) {
    if (!c) return fail(MINDIST_E_ARG, "ctx is NULL");
    if (m_full) *m_full = c->P.m_full;
    if (k_partial) *k_partial = c->P.k_m;
    if (n_gamma) *n_gamma = Schedule(c->P.k, c->P.m_full, c->P.k_m, c->partial_policy).n_sets();
    return MINDIST_OK;
}

// ---------------------------------------------------------------------------
// one pair of Algorithm 1 on the device
namespace {

constexpr int kDefaultBlocksPerCu = 4;

// Resident workgroups per CU the enumeration launches of set j's pairs are
// sized for: the option when set; else 4, or, for the matrix-core kernel
// (its products and operands hold up to 216 VGPRs), as many as its
// registers let one CU hold, at most 4.
int blocks_per_cu_for(const mindist_ctx *c, int j) {
    if (c->blocks_per_cu) return c->blocks_per_cu;
    const int D = c->gd[j].D;
    if (c->mfma && !c->verify && D <= kMfmaMaxD) {
        const int n = enum_mfma_resident_blocks(D, c->items);
        if (n >= 1) return std::min(n, kDefaultBlocksPerCu);
    }
    return kDefaultBlocksPerCu;
}


// Chunks of a pair.  Left tiles are runs of 64*items consecutive left
// subsets (colex order); a left tile whose first subset has largest element
// e pairs with C(k-1-e, b) right entries, cut into right tiles of T.
// groups[] lists the runs of left tiles sharing e (left-major order);
// rprefix[r] (right-major order) is the first chunk of right tile r, whose
// left tiles are the prefix of tiles that still have entries past r*T.
PairPlan plan_pair(const mindist_ctx *c, int j, int w, GroupEntry *groups,
                   std::vector<uint64_t> *rprefix) {
    const int k = c->P.k;
    const Binom &B = BN();
    PairPlan pp;
    const Split sp = choose_split(k, w, c->gd[j].bcap, false, c->min_items);
    pp.a = sp.a;
    pp.b = sp.b;
    pp.b2 = sp.b2;
    const uint64_t TB = 64ull * c->items;   // left subsets per tile
    pp.n_items = B(k - pp.b - pp.b2, pp.a);
    if (c->tile_t) {
        pp.T = c->tile_t;
    } else if (pp.b2 == 0) {
        // Right tile length from the exact chunk count at each candidate.  A
        // pair that fits one round of the resident waves (every chunk taken
        // by its wave at launch, no claims) is bound by the latency of one
        // wave's walk down its tile: the shortest tile that still fits one
        // round.  A larger pair is bound by throughput: the longest tile
        // (fewer chunk set-ups) that still leaves every wave max(2, D-1)
        // chunks, so the last chunks leave little idle time (a chunk takes
        // longer as D grows).  Measured per pair on D = 3 and D = 7 codes.
        const uint64_t waves = (uint64_t)c->cus * blocks_per_cu_for(c, j) * 4;
        // left tiles and right entries of each group, then chunks per T
        std::vector<std::pair<uint64_t, uint64_t>> grp;
        {
            const uint64_t tiles_ = ceil_div(pp.n_items, TB);
            for (int e = pp.a - 1; e <= k - 1 - pp.b; ++e) {
                const uint64_t lt_lo = ceil_div(B(e, pp.a), TB);
                const uint64_t lt_hi = std::min(ceil_div(B(e + 1, pp.a), TB), tiles_);
                if (lt_hi > lt_lo) grp.emplace_back(lt_hi - lt_lo, B(k - 1 - e, pp.b));
            }
        }
        auto chunks_at = [&](uint32_t T) {
            const int sh = __builtin_ctz(T);
            uint64_t n = 0;
            for (const auto &g : grp) n += g.first * ((g.second + T - 1) >> sh);
            return n;
        };
        uint32_t T = 0;
        for (uint32_t t = 16; t <= 256 && !T; t <<= 1)
            if (chunks_at(t) <= waves) T = t;
        if (!T) {
            const uint64_t per_wave = (uint64_t)std::max(2, c->gd[j].D - 1);
            T = 128;
            for (uint32_t t = 1024; t > 128; t >>= 1)
                if (chunks_at(t) >= per_wave * waves) { T = t; break; }
        }
        pp.T = T;
    } else {
        pp.T = outer_tile(k, sp, (uint32_t)TB);
    }
    const uint64_t tiles = ceil_div(pp.n_items, TB);
    uint64_t base = 0;
    std::vector<uint64_t> lt_end;
    for (int e = pp.a - 1; e <= k - 1 - pp.b - pp.b2; ++e) {
        const uint64_t lo = B(e, pp.a), hi = B(e + 1, pp.a);
        const uint64_t lt_lo = ceil_div(lo, TB), lt_hi = std::min(ceil_div(hi, TB), tiles);
        if (lt_hi <= lt_lo) continue;
        GroupEntry &g = groups[pp.ngroups++];
        g.chunk_base = base;
        g.lt_begin = lt_lo;
        g.nr_first = (uint32_t)B(k - 1 - pp.b2 - e, pp.b);
        g.n_rt = ceil_div(g.nr_first, pp.T);
        g.e = (uint32_t)e;
        base += (lt_hi - lt_lo) * g.n_rt;
        lt_end.push_back(lt_hi);
    }
    pp.total_chunks = base;
    if (rprefix) {
        // n_rt falls (weakly) from group to group, so the left tiles with
        // more than r right tiles are those of the groups with n_rt > r
        rprefix->clear();
        pp.n_rt = pp.ngroups ? (uint32_t)groups[0].n_rt : 0;
        uint64_t acc = 0;
        int gl = pp.ngroups - 1;
        for (uint32_t r = 0; r < pp.n_rt; ++r) {
            while (gl >= 0 && groups[gl].n_rt <= r) --gl;
            rprefix->push_back(acc);
            acc += lt_end[gl];
        }
        rprefix->push_back(acc);
    }
    return pp;
}

}  // namespace

static int run_impl(mindist_ctx *c, mindist_result *out) {
    if (!c || !out) return fail(MINDIST_E_ARG, "NULL argument");
    const auto t0 = std::chrono::steady_clock::now();
    const Plan &P = c->P;
    const int n = P.n, k = P.k;
    const Schedule S(k, P.m_full, P.k_m, c->partial_policy);
    const int ng = S.n_sets();
    const bool per_level = c->term_per_level != 0;
    const Binom &B = BN();
    std::memset(out, 0, sizeof(*out));
    c->trace.clear();
    c->have_run = false;
    if (launch_init_state(c->d_state, c->max_pairs, c->stream))
        return fail(MINDIST_E_HIP, "init kernel launch failed");
    if (c->noalloc && launch_fill_u32(reinterpret_cast<uint32_t *>(c->d_mail), 0u,
                                      kMailRing * sizeof(PairMail) / 4, c->stream))
        return fail(MINDIST_E_HIP, "mailbox clear failed");
    if (c->inject_u) {
        // testing: the device starts from a least weight it never found
        uint32_t *h = static_cast<uint32_t *>(pinned_alloc(sizeof(uint32_t)));
        if (!h) return fail(MINDIST_E_NOMEM, "inject_u staging");
        *h = c->inject_u;
        const bool ok =
            hipMemcpyAsync(&c->d_state->U_found, h, sizeof(uint32_t), hipMemcpyHostToDevice, c->stream) == hipSuccess &&
            hipMemcpyAsync(&c->d_state->U_base, h, sizeof(uint32_t), hipMemcpyHostToDevice, c->stream) == hipSuccess &&
            hipStreamSynchronize(c->stream) == hipSuccess;
        pinned_free(h);
        if (!ok) return fail(MINDIST_E_HIP, "inject_u copy failed");
    }

    const int singleton = n - k + 1;
    int L = 1;
    uint32_t U_found = kInf;
    int pairs = 0, exited = 0, last_j = -1, last_w = 0;
    uint64_t executed_total = 0, canonical_total = 0;
    double enum_s = 0;
    int launches = 0;
    const int midpair = c->midpair_exit && !c->term_per_level;
    int status = MINDIST_OK;

    // A pair ready to launch: its plan, chunk groups (device address) and
    // tables (built in stream order).
    struct Prep {
        int j = 0, w = 0;
        PairPlan pp;
        const GroupEntry *groups = nullptr;   // device copy (shared per shape)
        uint32_t *table = nullptr, *ltable = nullptr, *table2 = nullptr, *cnt2 = nullptr;
    };
    // per-wave totals: one entry per wave of the widest launch
    {
        const uint64_t max_waves = (uint64_t)c->cus * std::max(kDefaultBlocksPerCu, c->blocks_per_cu) * 4;
        if (max_waves > c->parts_cap && c->noalloc)
            return fail(MINDIST_E_LIMIT, "more resident waves than the fixed region holds");
        if (max_waves > c->parts_cap) {
            dev_free(c->d_parts);
            c->d_parts = static_cast<WavePart *>(dev_alloc(sizeof(WavePart) * max_waves));
            c->parts_cap = c->d_parts ? max_waves : 0;
            if (!c->d_parts) return fail(MINDIST_E_NOMEM, "per-wave buffer allocation failed");
        }
    }
    // The plan of pair (j, w) (cached per context) with the device copy of
    // its chunk groups.  Groups depend only on (k, a, b, b2, T, lane items),
    // so one copy per shape serves every context on the device.  In the
    // right-major order the plan also fills the host prefix table.
    std::vector<GroupEntry> plan_tmp(c->groups_cap);
    auto plan = [&](Prep &q, int j, int w) -> int {
        q.j = j;
        q.w = w;
        q.table = q.ltable = q.table2 = q.cnt2 = nullptr;
        const std::array<uint64_t, 6> key{(uint64_t)j << 32 | (uint32_t)w, (uint64_t)c->items,
                                          (uint64_t)c->tile_t, (uint64_t)c->blocks_per_cu,
                                          c->min_items, (uint64_t)c->order};
        if (c->noalloc) {
            // one pair in flight: its groups go to the fixed slot (the
            // previous pair has finished; a pageable copy has consumed
            // plan_tmp when it returns)
            q.pp = plan_pair(c, j, w, plan_tmp.data(), nullptr);
            if (hipMemcpyAsync(c->d_groups_fixed, plan_tmp.data(), sizeof(GroupEntry) * q.pp.ngroups,
                               hipMemcpyHostToDevice, c->stream) != hipSuccess)
                return fail(MINDIST_E_HIP, "chunk group upload failed");
            q.groups = c->d_groups_fixed;
            return MINDIST_OK;
        }
        if (!c->order) {
            auto it = c->plan_cache.find(key);
            if (it != c->plan_cache.end()) {
                q.pp = it->second.first;
                q.groups = it->second.second;
                return MINDIST_OK;
            }
        }
        q.pp = plan_pair(c, j, w, plan_tmp.data(), c->order ? &c->rprefix_host : nullptr);
        const uint32_t shape[6] = {(uint32_t)k, (uint32_t)q.pp.a, (uint32_t)q.pp.b, (uint32_t)q.pp.b2,
                                   q.pp.T, (uint32_t)c->items};
        q.groups = static_cast<const GroupEntry *>(
            device_const(shape, sizeof(shape), plan_tmp.data(), sizeof(GroupEntry) * q.pp.ngroups));
        if (!q.groups) return fail(MINDIST_E_NOMEM, "chunk group upload failed");
        if (!c->order) c->plan_cache.emplace(key, std::make_pair(q.pp, q.groups));
        return MINDIST_OK;
    };
    // tables of a planned pair (built in stream order on first use)
    auto stage = [&](Prep &q) -> int {
        if (c->noalloc) {
            // tables of one pair at a time, rebuilt in the arena
            for (auto &g : c->gd) g.tabs.clear();
            c->arena_used = 0;
        }
        int e = get_table(c, q.j, q.pp.b, 1, q.pp.b2, &q.table, &q.cnt2);
        if (e) return e;
        if (q.pp.b2) {
            e = get_table(c, q.j, q.pp.b2, 1, 0, &q.table2);
            if (e) return e;
        }
        if (c->left_tables && left_table_fits(c, q.j, q.pp.a)) {
            e = get_table(c, q.j, q.pp.a, 0, 0, &q.ltable);
            if (e) return e;
        }
        return MINDIST_OK;
    };
    // the right-major order's prefix table is uploaded right before its launch
    auto upload_rprefix = [&]() -> int {
        std::vector<uint64_t> &rpre = c->rprefix_host;
        if (rpre.size() > c->rprefix_cap) {
            dev_free(c->d_rprefix);
            pinned_free(c->h_rprefix);
            c->rprefix_cap = std::max<size_t>(rpre.size(), 2 * c->rprefix_cap);
            c->d_rprefix = static_cast<uint64_t *>(dev_alloc(c->rprefix_cap * 8));
            c->h_rprefix = static_cast<uint64_t *>(pinned_alloc(c->rprefix_cap * 8));
            if (!c->d_rprefix || !c->h_rprefix) {
                c->rprefix_cap = 0;
                return fail(MINDIST_E_NOMEM, "chunk-order table allocation failed");
            }
        }
        std::memcpy(c->h_rprefix, rpre.data(), rpre.size() * 8);
        if (hipMemcpyAsync(c->d_rprefix, c->h_rprefix, rpre.size() * 8, hipMemcpyHostToDevice,
                           c->stream) != hipSuccess)
            return fail(MINDIST_E_HIP, "chunk-order table upload failed");
        return MINDIST_OK;
    };
    // wait for the mailbox of pair `pr` (the publish kernel behind it fills it)
    auto wait_mail = [&](int pr) -> int {
        if (c->noalloc) {
            PairMail *h = &c->h_mail[pr % kMailRing];
            HIPCHK(hipMemcpyAsync(h, &c->d_mail[pr % kMailRing], sizeof(PairMail), hipMemcpyDeviceToHost,
                                  c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
            if (h->seq != (uint32_t)pr + 1)
                return fail(MINDIST_E_HIP, "enumeration kernel ended without publishing its pair");
            return MINDIST_OK;
        }
        const uint32_t *seq = &c->h_mail[pr % kMailRing].seq;
        std::chrono::steady_clock::time_point idle_since{};
        bool idle = false;
        for (uint64_t spin = 1;; ++spin) {
            if (__atomic_load_n(seq, __ATOMIC_ACQUIRE) == (uint32_t)pr + 1) return MINDIST_OK;
            if ((spin & 255) == 0) {
                const hipError_t q = hipStreamQuery(c->stream);
                if (q != hipSuccess && q != hipErrorNotReady)
                    return fail(MINDIST_E_HIP, std::string("enumeration kernel failed: ") + hipGetErrorString(q));
                if (q == hipSuccess) {
                    // the stream can report completion before the kernel's
                    // last write to host memory has landed: allow it a moment
                    const auto now = std::chrono::steady_clock::now();
                    if (!idle) { idle = true; idle_since = now; }
                    else if (now - idle_since > std::chrono::milliseconds(50))
                        return fail(MINDIST_E_HIP, "enumeration kernel ended without publishing its pair");
                }
            }
            __builtin_ia32_pause();
        }
    };
    if (c->profile) {
        while (c->pair_ev.size() < (size_t)2 * c->max_pairs) {
            hipEvent_t e = event_get();
            if (!e) return fail(MINDIST_E_HIP, "event creation failed");
            c->pair_ev.push_back(e);
        }
    }

    // A pair ready to run as pair index idx with bound L_prev.
    struct Flight { Prep q; PairPos pos; int idx = 0; int L_prev = 0; int blocks = 0; };
    auto blocks_of = [&](const Prep &q) {
        const uint64_t want = ceil_div(q.pp.total_chunks, 4);
        return (int)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)c->cus * blocks_per_cu_for(c, q.j)));
    };
    // the plan of every pair launched in this run (a witness may come from a
    // pair launched but not visited, in a launch shared with visited ones)
    std::vector<Flight> launched_pairs;
    std::vector<int> leader;          // profile: the first pair of each pair's launch
    // Launch staged pairs (consecutive indices, same D) as one kernel, and
    // the kernel that publishes their results behind it.
    auto launch = [&](const std::vector<Flight> &grp) -> int {
        GroupArgs ga{};
        ga.n = (uint32_t)grp.size();
        uint32_t bs = 0;
        for (size_t t = 0; t < grp.size(); ++t) {
            const Prep &q = grp[t].q;
            const GammaDev &g = c->gd[q.j];
            const PairPlan &pp = q.pp;
            PairArgs &pa = ga.p[t];
            pa.rows = g.rows;
            pa.table = q.table;
            pa.ltable = q.ltable;
            pa.binom = c->d_binom;
            pa.groups = q.groups;
            pa.st = c->d_state;
            pa.n_items = pp.n_items;
            pa.total_chunks = pp.total_chunks;
            pa.cancel_after = c->cancel_after;
            pa.ngroups = pp.ngroups;
            pa.k = k;
            pa.a = pp.a;
            pa.b = pp.b;
            pa.b2 = pp.b2;
            pa.table2 = q.table2;
            pa.cnt2 = q.cnt2;
            pa.T = pp.T;
            pa.offset = g.stripped ? (uint32_t)q.w : 0u;
            pa.L_prev = (uint32_t)grp[t].L_prev;
            pa.pair = (uint32_t)grp[t].idx;
            pa.midpair_exit = (uint32_t)midpair;
            pa.max_pairs = c->max_pairs;
            pa.rprefix = c->d_rprefix;
            pa.order = (uint32_t)c->order;
            pa.n_rt = pp.n_rt;
            pa.counters = (uint32_t)c->counters;
            pa.waves = (uint32_t)grp[t].blocks * 4u;
            pa.parts = c->d_parts + (size_t)bs * 4;
            ga.block_start[t] = bs;
            bs += (uint32_t)grp[t].blocks;
            if (!c->noalloc) __atomic_store_n(&c->h_mail[grp[t].idx % kMailRing].seq, 0u, __ATOMIC_RELEASE);
            launched_pairs.push_back(grp[t]);
            leader.push_back(grp[0].idx);
        }
        ga.block_start[grp.size()] = bs;
        if ((uint64_t)bs * 4 > c->parts_cap) return fail(MINDIST_E_HIP, "launch exceeds the per-wave buffer");
        const int idx0 = grp[0].idx;
        if (c->profile && hipEventRecord(c->pair_ev[2 * idx0], c->stream) != hipSuccess)
            return fail(MINDIST_E_HIP, "event record failed");
        if (launch_enum_pair(ga, c->gd[grp[0].q.j].D, c->items, c->verify, c->mfma, c->stream))
            return fail(MINDIST_E_HIP, "enumeration kernel launch failed");
        if (c->profile && hipEventRecord(c->pair_ev[2 * idx0 + 1], c->stream) != hipSuccess)
            return fail(MINDIST_E_HIP, "event record failed");
        if (launch_publish_pair(ga, c->d_mail, c->stream))
            return fail(MINDIST_E_HIP, "publish kernel launch failed");
        ++launches;
        return MINDIST_OK;
    };
    auto beyond_limit = [&](int w) { return w > MINDIST_MAX_LEVEL || B(k, w) >= (1ull << 63); };

    // Pairs run in Algorithm 1's order.  The pair Algorithm 1 visits next is
    // launched once its test passes; behind it, further pairs are launched
    // ahead of their results (with the bound they get if every pair before
    // them completes) while the work already queued is small, so the device
    // never waits for the host between short pairs.  Short consecutive pairs
    // of the same width share one launch (block ranges per pair), as long as
    // all their blocks fit one round of the resident ones.  If Algorithm 1
    // stops, the pairs launched ahead read U <= their bound and leave at once
    // (with mid-pair exit on; otherwise only one pair of at most `speculate`
    // combinations is launched ahead, and no launch is shared).
    std::deque<Flight> fl;          // launched, not read yet; front: next pair visited
    PairPos npos = S.first();       // the next pair to launch
    bool nmore = true;              // npos is a pair of the schedule
    int L_pred = L;                 // the bound before it
    int next_idx = 0;
    PairMail last_mail{};
    const bool free_exit = midpair && !c->deadline_ms;
    const bool grouping = free_exit && c->speculate && !c->order && !c->cancel_after;
    constexpr uint64_t kAheadWork = 1ull << 30;   // queued combinations that stop a second launch ahead
    // Stage pair npos as index next_idx with bound L0, extend the launch
    // with the following short pairs when allowed, launch, and queue them.
    auto launch_from_next = [&](int L0, bool may_group) -> int {
        std::vector<Flight> grp;
        int L_cur = L0;
        int blocks = 0;
        for (;;) {
            Flight f;
            f.pos = npos;
            int e = plan(f.q, npos.j, npos.h);
            if (e) return e;
            f.blocks = blocks_of(f.q);
            if (!grp.empty()) {
                // joins the launch only if it is short and of the same width
                const bool ok = f.q.pp.b2 == 0 && grp[0].q.pp.b2 == 0 &&
                                c->gd[npos.j].D == c->gd[grp[0].q.j].D &&
                                (uint64_t)f.q.pp.total_chunks <= 4ull * (uint64_t)f.blocks &&
                                blocks + f.blocks <= c->cus * blocks_per_cu_for(c, grp[0].q.j);
                if (!ok) break;
            }
            e = stage(f.q);
            if (e) return e;
            if (grp.empty() && c->order) {
                e = upload_rprefix();
                if (e) return e;
            }
            f.idx = next_idx++;
            f.L_prev = L_cur;
            blocks += f.blocks;
            grp.push_back(f);
            L_cur = S.L_after(npos, per_level, L_cur);
            L_pred = L_cur;
            nmore = S.next(npos, &npos);
            const bool first_short = (uint64_t)grp[0].q.pp.total_chunks <= 4ull * (uint64_t)grp[0].blocks;
            if (!may_group || !grouping || !first_short || (int)grp.size() >= kGroupMax ||
                fl.size() + grp.size() >= (size_t)kMailRing - 1 || !nmore || beyond_limit(npos.h) ||
                next_idx >= c->max_pairs ||
                L_cur >= (int)std::min<uint32_t>(U_found, (uint32_t)singleton))
                break;
        }
        int e = launch(grp);
        if (e) return e;
        for (auto &f : grp) fl.push_back(f);
        return MINDIST_OK;
    };
    for (bool more = ng >= 1 && k >= 1; more;) {
        const PairPos pos = fl.empty() ? npos : fl.front().pos;
        const int j = pos.j, w = pos.h;
        const int U = (int)std::min<uint32_t>(U_found, (uint32_t)singleton);
        // Algorithm 1's test: before every pair (per-pair rule) or before a
        // level (literal per-level rule)
        if (L >= U && (!per_level || S.level_start(pos))) break;
        if (beyond_limit(w)) {
            status = fail(MINDIST_E_LIMIT, "pair (" + std::to_string(j) + "," + std::to_string(w) +
                                               ") exceeds the rank-space limit");
            break;
        }
        if (c->deadline_ms) {
            const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (el * 1000.0 > (double)c->deadline_ms) {
                status = fail(MINDIST_E_TIMEOUT, "deadline reached");
                break;
            }
        }
        if (fl.empty()) {
            int e = launch_from_next(L, true);
            if (e) return e;
        }
        // launch ahead
        // (not once the U already known is at or below the pair's bound:
        // Algorithm 1 certainly stops before it)
        while (c->speculate && !c->cancel_after && !c->order && fl.size() < (size_t)kMailRing - 1 &&
               nmore && !beyond_limit(npos.h) && next_idx < c->max_pairs &&
               L_pred < (int)std::min<uint32_t>(U_found, (uint32_t)singleton)) {
            uint64_t queued = 0;
            for (const Flight &x : fl) queued += B(k, x.q.w);
            // one pair ahead always; more only while the queued work is short
            if (free_exit ? (fl.size() >= 2 && queued >= kAheadWork)
                          : (fl.size() >= 2 || B(k, npos.h) > c->speculate))
                break;
            int e = launch_from_next(L_pred, true);
            if (e) return e;
        }
        const Flight f = fl.front();
        fl.pop_front();
        int e = wait_mail(f.idx);
        if (e) return e;
        const GammaDev &g = c->gd[j];
        const PairPlan &pp = f.q.pp;
        const PairMail hm = c->h_mail[f.idx % kMailRing];
        last_mail = hm;
        // U after this pair: the least weight of the pairs visited so far (the
        // device's U_found may already hold a later pair of a shared launch)
        U_found = std::min(U_found, hm.pair_min);
        const int Lb = L;
        const bool cut = midpair && hm.executed < B(k, w) && !hm.cancelled;
        if (!cut) L = S.L_after(pos, per_level, L);
        mindist_pair rec{};
        rec.j = j; rec.w = w; rec.L_before = Lb; rec.L_after = L;
        rec.U_after = (int)std::min<uint32_t>(U_found, (uint32_t)singleton);
        rec.pair_min = hm.pair_min == kInf ? -1 : (int)hm.pair_min;
        rec.count = B(k, w);
        rec.executed = hm.executed;
        rec.wsum = hm.wsum;
        rec.dwords = g.D;
        rec.split_a = pp.a;
        rec.split_b = pp.b;
        rec.split_b2 = pp.b2;
        rec.dev_ms = hm.t_end > hm.t_begin ? (double)(hm.t_end - hm.t_begin) / c->wall_hz * 1e3 : 0.0;
        rec.launch = leader[f.idx];
        c->trace.push_back(rec);
        executed_total += hm.executed;
        canonical_total += rec.count;
        ++pairs;
        last_j = j;
        last_w = w;
        if (hm.cancelled) { status = fail(MINDIST_E_CANCELLED, "cancelled after the chunk budget"); break; }
        // the kernels stop a pair only once the least weight they know (from
        // earlier launches and earlier pairs of this one) is at or below the
        // bound before it; the certificate below checks that the host's own
        // U -- the least pair minimum up to this pair -- justifies the cut
        if (cut) { exited = 1; break; }
        PairPos nx;
        if (!S.next(pos, &nx)) break;
    }
    // pairs launched ahead of a stop still run (they find nothing below U
    // and leave at once): return with the stream idle
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->profile && pairs) {
        for (int t = 0; t < pairs; ++t) {
            // pairs of a shared launch report that launch's time
            float ms = 0, t_ms = 0;
            const int l = leader[t];
            HIPCHK(hipEventElapsedTime(&ms, c->pair_ev[2 * l], c->pair_ev[2 * l + 1]));
            HIPCHK(hipEventElapsedTime(&t_ms, c->pair_ev[0], c->pair_ev[2 * l]));
            c->trace[t].ms = ms;
            c->trace[t].t_start_ms = t_ms;
            if (l == t) enum_s += ms * 1e-3;
        }
    }
    out->n = n;
    out->k = k;
    out->m_full = P.m_full;
    out->k_partial = P.k_m;
    out->n_gamma = ng;
    out->U_found = U_found == kInf ? n + 1 : (int)U_found;
    out->d = (int)std::min<uint32_t>(U_found, (uint32_t)singleton);
    out->L_final = L;
    out->pairs_visited = pairs;
    out->exited_midpair = exited;
    out->w_last = last_w;
    out->j_last = last_j;
    out->executed_total = executed_total;
    out->canonical_total = canonical_total;
    out->seconds_enum = enum_s;
    out->enum_launches = launches;
    if (status != MINDIST_OK) {
        out->seconds_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return status;
    }
    {
        CertSpec cs;
        cs.n = n;
        cs.k = k;
        cs.sched = S;
        cs.per_level = per_level;
        cs.midpair_exit = midpair != 0;
        std::vector<PairView> views(c->trace.size());
        for (size_t t = 0; t < views.size(); ++t) views[t] = view_of(c->trace[t]);
        const int e = certify_trace(cs, views.data(), (int)views.size(), out->d, out->L_final,
                                    out->exited_midpair);
        if (e) return e;
    }
    // witness: slot[U_found], written by the wave that first lowered the
    // device's U_found to it, normally reaches the host in the mailbox of the
    // last pair read; it may come from a pair launched with the visited ones
    // but not visited itself (any codeword of weight U_found will do)
    if (U_found != kInf) {
        Slot s = last_mail.witness;
        if (last_mail.U_found != U_found) {
            // a pair launched but not visited found a lower weight (possible
            // only when the Singleton bound ends the run): read slot[U_found]
            Slot host_slot{};
            Slot *h = c->noalloc ? &host_slot : static_cast<Slot *>(pinned_alloc(sizeof(Slot)));
            if (!h) return fail(MINDIST_E_NOMEM, "witness readback allocation failed");
            const bool ok = hipMemcpyAsync(h, state_slots(c->d_state) + U_found, sizeof(Slot),
                                           hipMemcpyDeviceToHost, c->stream) == hipSuccess &&
                            hipStreamSynchronize(c->stream) == hipSuccess;
            s = *h;
            if (!c->noalloc) pinned_free(h);
            if (!ok) return fail(MINDIST_E_HIP, "witness readback failed");
        }
        if (s.pair >= (uint32_t)launched_pairs.size())
            return fail(MINDIST_E_CERT, "witness slot holds an invalid pair index");
        const Flight &lp = launched_pairs[s.pair];
        const std::vector<int> rows = witness_rows(k, lp.q.pp.a, lp.q.pp.b, lp.q.pp.b2, s);
        const int e = certify_witness(P, lp.q.j, rows, lp.q.w, (int)U_found, out->witness,
                                      out->witness_rows);
        if (e) return e;
        out->witness_j = lp.q.j;
        out->witness_w = lp.q.w;
    }
    out->seconds_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    c->have_run = true;
    return MINDIST_OK;
}

extern "C" int mindist_run(mindist_ctx *c, mindist_result *out) {
    const int e = run_impl(c, out);
    // no launch of a run may outlive it: the next run reuses its mailboxes
    // (a stale publish could otherwise land in one it waits on)
    if (e != MINDIST_OK && c && c->stream) (void)hipStreamSynchronize(c->stream);
    return e;
}

namespace md {

// Fixed-region layout of mindist_run_noalloc (offsets 256-byte aligned):
// binomial table, run state, mailboxes, per-wave totals, the current pair's
// chunk groups, the rows of every Gamma_j, then the table arena.
// pairs of one run: n_gamma * min(k, 64) + 1 with n_gamma <= n/k + 1, at most
// n + k + 1 <= 577 for k <= 64 and 8 * 64 + 1 for k > 64
constexpr int kNoallocMaxPairs = 640;
constexpr uint64_t kNoallocMaxWaves = 256 * 4 * 4;
constexpr uint64_t kNoallocRowBytes = 256 * 1024;

static uint64_t a256(uint64_t x) { return (x + 255) & ~255ull; }

int noalloc_run(unsigned char *base, uint64_t bytes, bool *binom_ready, const uint64_t *G, int n, int k,
                hipStream_t stream, mindist_result *out, mindist_pair *pairs, int cap, int *n_pairs) {
    if (!out || (cap > 0 && !pairs) || cap < 0) return fail(MINDIST_E_ARG, "NULL argument");
    if (n_pairs) *n_pairs = 0;
    mindist_ctx *c = new (std::nothrow) mindist_ctx();   // host memory only
    if (!c) return fail(MINDIST_E_NOMEM, "context allocation failed");
    std::unique_ptr<mindist_ctx, void (*)(mindist_ctx *)> hold(c, free_ctx);
    int e = make_plan(G, n, k, c->P);
    if (e) return e;
    const Plan &P = c->P;
    c->noalloc = 1;
    c->stream = stream;
    c->own_stream = false;
    c->speculate = 0;        // one pair in flight: its tables and groups own the region
    c->left_tables = 0;      // lanes unrank their left subsets
    c->n_gamma = (int)P.sets.size();
    c->max_pairs = c->n_gamma * std::min(k, MINDIST_MAX_LEVEL) + 1;
    if (c->max_pairs > kNoallocMaxPairs) return fail(MINDIST_E_LIMIT, "too many pairs for the fixed region");
    HIPCHK(hipGetDevice(&c->device));
    HIPCHK(hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device));
    {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device) == hipSuccess && khz > 0)
            c->wall_hz = khz * 1000.0;
    }
    // carve the region
    uint64_t off = 0;
    auto take = [&](uint64_t sz) { unsigned char *p = base + off; off = a256(off + sz); return p; };
    const size_t binom_bytes = BN().t.size() * sizeof(uint64_t);
    c->d_binom = reinterpret_cast<const uint64_t *>(take(binom_bytes));
    c->d_state = reinterpret_cast<DevState *>(take(state_bytes(kNoallocMaxPairs)));
    c->d_mail = reinterpret_cast<PairMail *>(take(kMailRing * sizeof(PairMail)));
    c->d_parts = reinterpret_cast<WavePart *>(take(kNoallocMaxWaves * sizeof(WavePart)));
    c->parts_cap = kNoallocMaxWaves;
    c->groups_cap = k + 2;
    c->d_groups_fixed = reinterpret_cast<GroupEntry *>(take((uint64_t)(kBinomX + 2) * sizeof(GroupEntry)));
    unsigned char *rows = take(kNoallocRowBytes);
    c->arena = base + off;
    if (off >= bytes) return fail(MINDIST_E_LIMIT, "fixed region too small");
    c->arena_bytes = bytes - off;
    c->mail_host.assign(kMailRing, PairMail{});
    c->h_mail = c->mail_host.data();
    if (!*binom_ready) {
        // constant for every call on the device: uploaded once
        HIPCHK(hipMemcpyAsync(const_cast<uint64_t *>(c->d_binom), BN().t.data(), binom_bytes,
                              hipMemcpyHostToDevice, stream));
        HIPCHK(hipStreamSynchronize(stream));
        *binom_ready = true;
    }
    // Gamma rows (packed carried columns) and each set's table level cap: the
    // levels 1..b of one table within a quarter of the arena, so a pair's
    // tables (two-level: levels 1..b; three-level: the outer table with its
    // counts and the inner levels 1..b2) always fit
    const Binom &B = BN();
    c->gd.resize(c->n_gamma);
    std::vector<uint32_t> hrows;
    uint64_t roff = 0;
    for (int j = 0; j < c->n_gamma; ++j) {
        GammaDev &g = c->gd[j];
        const std::vector<int> cols = carried_columns(P, j);
        g.stripped = j < P.m_full;
        g.D = (int)((cols.size() + 31) / 32);
        g.DP = dp_of_host(g.D);
        const uint64_t words = (uint64_t)k * g.DP;
        if (a256(roff + words * 4) > kNoallocRowBytes)
            return fail(MINDIST_E_LIMIT, "Gamma rows exceed the fixed region");
        g.rows = reinterpret_cast<uint32_t *>(rows + roff);
        roff = a256(roff + words * 4);
        hrows.assign(words, 0);
        for (int r = 0; r < k; ++r) pack_row(&P.gamma[j][(size_t)r * P.W], cols, &hrows[(size_t)r * g.DP], g.DP);
        HIPCHK(hipMemcpyAsync(g.rows, hrows.data(), words * 4, hipMemcpyHostToDevice, stream));
        g.bcap = 0;
        uint64_t levels = 0;
        for (int b = 1; b <= 16 && b <= k; ++b) {
            const uint64_t ent = B(k, b);
            levels += ent * g.DP * 4 + 256;
            if (ent >= (1ull << 31) || levels > c->arena_bytes / 4) break;
            g.bcap = b;
        }
    }
    c->table_cap = c->arena_bytes / 4;
    e = run_impl(c, out);
    if (e != MINDIST_OK) (void)hipStreamSynchronize(stream);
    if (n_pairs) *n_pairs = (int)c->trace.size();
    for (int t = 0; t < cap && t < (int)c->trace.size(); ++t) pairs[t] = c->trace[t];
    return e;
}

}  // namespace md

extern "C" int mindist_get_pairs(const mindist_ctx *c, mindist_pair *out, int cap, int *n_out) {
    if (!c || (!out && cap > 0) || !n_out) return fail(MINDIST_E_ARG, "NULL argument");
    const int n = (int)c->trace.size();
    for (int i = 0; i < n && i < cap; ++i) out[i] = c->trace[i];
    *n_out = n;
    return MINDIST_OK;
}

extern "C" int mindist_calibrate(int dwords, int blocks_per_cu, double *codewords_per_s,
                                 double *seconds) {
    if (!codewords_per_s || !(dwords == 1 || dwords == 2 || dwords == 3 || dwords == 4 ||
                              dwords == 7 || dwords == 8) || blocks_per_cu < 1 || blocks_per_cu > 64)
        return fail(MINDIST_E_ARG, "calibrate: dwords in {1,2,3,4,7,8}, 1 <= blocks_per_cu <= 64");
    int dev = 0;
    hipDeviceProp_t prop;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    const int blocks = prop.multiProcessorCount * blocks_per_cu;
    const int dp = dwords <= 1 ? 1 : dwords <= 2 ? 2 : dwords <= 4 ? 4 : 8;
    std::vector<uint32_t> h(64 * dp);
    for (size_t i = 0; i < h.size(); ++i) h[i] = (uint32_t)(i * 2654435761u) ^ 0x5bd1e995u;
    uint32_t *tab = static_cast<uint32_t *>(dev_alloc(h.size() * 4));
    uint32_t *out = static_cast<uint32_t *>(dev_alloc((size_t)blocks * 256 * 4));
    hipStream_t s = stream_get();
    hipEvent_t e0 = event_get(), e1 = event_get();
    int rc = MINDIST_OK;
    if (!tab || !out || !s || !e0 || !e1) rc = fail(MINDIST_E_NOMEM, "calibrate: allocation failed");
    const uint32_t steps = 1u << 16;
    float ms = 0;
    if (rc == MINDIST_OK && (hipMemcpy(tab, h.data(), h.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
                             launch_peak(tab, 1024, out, dwords, blocks, s) ||       // warm-up
                             hipEventRecord(e0, s) != hipSuccess ||
                             launch_peak(tab, steps, out, dwords, blocks, s) ||
                             hipEventRecord(e1, s) != hipSuccess ||
                             hipEventSynchronize(e1) != hipSuccess ||
                             hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = fail(MINDIST_E_HIP, "calibrate: kernel failed");
    if (rc == MINDIST_OK) {
        const double cw = (double)blocks * 256 * 4 * steps;   // 4 lane items per step
        *codewords_per_s = cw / (ms * 1e-3);
        if (seconds) *seconds = ms * 1e-3;
    }
    dev_free(tab);
    dev_free(out);
    stream_put(s);
    event_put(e0);
    event_put(e1);
    return rc;
}

extern "C" int mindist_peak_xorpop(int variant, int blocks_per_cu, double *ops_per_s, double *seconds) {
    int items = 0, words = 0;
    if (!ops_per_s || blocks_per_cu < 1 || blocks_per_cu > 16 || peak_reg_shape(variant, &items, &words))
        return fail(MINDIST_E_ARG, "peak: variant 0..3, 1 <= blocks_per_cu <= 16, ops_per_s not NULL");
    int dev = 0, cus = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int blocks = cus * blocks_per_cu;
    uint32_t *out = static_cast<uint32_t *>(dev_alloc((size_t)blocks * 256 * 4));
    hipStream_t s = stream_get();
    hipEvent_t e0 = event_get(), e1 = event_get();
    int rc = MINDIST_OK;
    if (!out || !s || !e0 || !e1) rc = fail(MINDIST_E_NOMEM, "peak: allocation failed");
    // about 25-100 ms per launch at 4-16 blocks per CU
    const uint32_t steps = ((1u << 19) / (uint32_t)(items * words)) & ~3u;
    float best = 0;
    for (int rep = 0; rc == MINDIST_OK && rep < 4; ++rep) {
        float ms = 0;
        // the first launch warms the clock and the code object up
        if (hipEventRecord(e0, s) != hipSuccess ||
            launch_peak_reg(variant, steps, 0x1234567u + rep, out, blocks, s) ||
            hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = fail(MINDIST_E_HIP, "peak: kernel failed");
            break;
        }
        if (rep > 0 && (best == 0 || ms < best)) best = ms;
    }
    if (rc == MINDIST_OK) {
        const double ops = (double)blocks * 256 * steps * items * words;
        *ops_per_s = ops / (best * 1e-3);
        if (seconds) *seconds = best * 1e-3;
    }
    dev_free(out);
    if (s) stream_put(s);
    event_put(e0);
    event_put(e1);
    return rc;
}

extern "C" int mindist_walk_pair(mindist_ctx *c, int j, int w, int blocks_per_cu, int32_t *pair_min,
                                 uint64_t *executed, double *seconds) {
    if (!c || !pair_min) return fail(MINDIST_E_ARG, "NULL argument");
    if (j < 0 || j >= c->n_gamma) return fail(MINDIST_E_ARG, "walk: no such information set");
    const GammaDev &g = c->gd[j];
    const int k = c->P.k;
    if (w < 1 || w > k) return fail(MINDIST_E_ARG, "walk: need 1 <= w <= k");
    if (w > kWalkMaxW || k > kWalkMaxK || g.D > kWalkMaxD)
        return fail(MINDIST_E_LIMIT, "walk: needs w <= 12, k <= 128 and at most 4 carried words");
    if (blocks_per_cu < 0 || blocks_per_cu > 16) return fail(MINDIST_E_ARG, "walk: blocks_per_cu in 0..16");
    const int bpc = blocks_per_cu > 0 ? blocks_per_cu : 4;
    const uint64_t total = BN()(k, w);
    const uint64_t threads = (uint64_t)c->cus * bpc * 256;
    WalkArgs a{};
    a.rows = g.rows;
    a.binom = c->d_binom;
    a.total = total;
    a.per_thread = ceil_div(total, threads);
    a.k = k;
    a.w = w;
    a.offset = g.stripped ? (uint32_t)w : 0u;
    a.out = static_cast<WalkOut *>(dev_alloc(sizeof(WalkOut)));
    hipEvent_t e0 = event_get(), e1 = event_get();
    WalkOut res{kInf, 0, 0};
    int rc = MINDIST_OK;
    float ms = 0;
    if (!a.out || !e0 || !e1) rc = fail(MINDIST_E_NOMEM, "walk: allocation failed");
    if (rc == MINDIST_OK &&
        (hipMemcpyAsync(a.out, &res, sizeof(res), hipMemcpyHostToDevice, c->stream) != hipSuccess ||
         hipEventRecord(e0, c->stream) != hipSuccess ||
         launch_walk_pair(a, g.D, c->cus * bpc, c->stream) != 0 ||
         hipEventRecord(e1, c->stream) != hipSuccess ||
         hipMemcpyAsync(&res, a.out, sizeof(res), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
         hipStreamSynchronize(c->stream) != hipSuccess ||
         hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        rc = fail(MINDIST_E_HIP, "walk: kernel failed");
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    dev_free(a.out);
    event_put(e0);
    event_put(e1);
    if (rc) return rc;
    *pair_min = res.min_weight == kInf ? -1 : (int32_t)res.min_weight;
    if (executed) *executed = res.executed;
    if (seconds) *seconds = ms * 1e-3;
    return MINDIST_OK;
}

extern "C" int mindist_device(char *name, int cap, int *compute_units) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return md::fail(MINDIST_E_HIP, "no HIP device");
    if (name && cap > 0) {
        std::strncpy(name, prop.gcnArchName, (size_t)cap - 1);
        name[cap - 1] = 0;
    }
    if (compute_units) *compute_units = prop.multiProcessorCount;
    return MINDIST_OK;
}
