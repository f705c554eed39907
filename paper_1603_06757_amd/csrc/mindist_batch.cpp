// mindist_batch.cpp -- host side of the persistent multi-code path:
// preprocessing of many codes (a thread pool runs the information-set
// partition and packing), the device layout of code slots, the launch (as
// one captured hipGraph: uploads + persistent kernel), and decoding of the
// per-code results.  The server reuses the engine with slots that are
// refilled between launches.
#include "mindist_batch_engine.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>

#include "../../include/mindist.h"
#include "mindist_plan.h"
#include "mindist_pool.h"

namespace md {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t job_bytes(int k) {
    const size_t b = sizeof(BatchJob) + sizeof(GroupEntry) * (size_t)(k + 2);
    return (b + 127) / 128 * 128;
}

// Largest level w Algorithm 1 is expected to reach on a random [n,k] code:
// the pair sequence's lower bound against the Gilbert-Varshamov distance
// (smallest d with sum_{i<=d} C(n,i) >= 2^(n-k)) plus a margin of two.
// It only sizes the saved tables: pairs beyond it still run, with the
// tables that exist.
static int expected_top_level(const HostCode &hc) {
    const int n = hc.n, k = hc.k;
    auto log2c = [](int a, int b) {
        return (std::lgamma(a + 1.0) - std::lgamma(b + 1.0) - std::lgamma(a - b + 1.0)) / std::log(2.0);
    };
    double acc = -1e300;          // log2 of the partial sum
    int d = n - k + 1;
    for (int i = 0; i <= n; ++i) {
        const double t = log2c(n, i);
        acc = acc > t ? acc + std::log2(1.0 + std::exp2(t - acc)) : t + std::log2(1.0 + std::exp2(acc - t));
        if (acc >= n - k) { d = i; break; }
    }
    d = std::min(d + 2, n - k + 1);
    int top = 1, L = 1;
    for (int w = 1; w <= k; ++w)
        for (int j = 0; j < hc.n_gamma; ++j) {
            if (L >= d) return top;
            top = w;
            L = bound_after(k, hc.P.m_full, hc.P.k_m, hc.n_gamma, j, w);
        }
    return top;
}

// Combinations Algorithm 1 is expected to enumerate: every pair in order
// while the bound is below a Gilbert-Varshamov estimate of d (the least w
// with sum_{i<=w} C(n,i) >= 2^(n-k)).
double estimated_work(const HostCode &hc) {
    const int n = hc.n, k = hc.k;
    auto log2c = [](int a, int b) {
        return (std::lgamma(a + 1.0) - std::lgamma(b + 1.0) - std::lgamma(a - b + 1.0)) / std::log(2.0);
    };
    double acc = -1e300;
    int d = n - k + 1;
    for (int i = 0; i <= n; ++i) {
        const double t = log2c(n, i);
        acc = acc > t ? acc + std::log2(1.0 + std::exp2(t - acc)) : t + std::log2(1.0 + std::exp2(acc - t));
        if (acc >= n - k) { d = i; break; }
    }
    double work = 0;
    int L = 1;
    for (int w = 1; w <= k; ++w)
        for (int j = 0; j < hc.n_gamma; ++j) {
            if (L >= d) return work;
            work += std::exp2(log2c(k, w));
            L = bound_after(k, hc.P.m_full, hc.P.k_m, hc.n_gamma, j, w);
        }
    return work;
}

int single_path_bytes(const uint64_t *G, int n, int k, uint64_t table_cap, size_t &bytes) {
    HostCode hc;
    hc.n = n;
    hc.k = k;
    int e = make_plan(G, n, k, hc.P);
    if (e) return e;
    hc.n_gamma = (int)hc.P.sets.size();
    const Binom &B = BN();
    // saved sums of s-subsets up to ceil(top / 2) for the expected top level
    // (the balanced split's right and left sizes), each only if it fits the
    // table cap
    const int smax = (expected_top_level(hc) + 1) / 2;
    bytes = (size_t)1 << 20;          // run state, per-wave totals, mailboxes
    for (int j = 0; j < hc.n_gamma; ++j) {
        const int dp = dp_of_host((int)((carried_columns(hc.P, j).size() + 31) / 32));
        bytes += align256((size_t)k * dp * 4);
        for (int sz = 1; sz <= smax && sz <= k; ++sz) {
            const uint64_t tb = B(k, sz) * (uint64_t)dp * 4;
            if (tb > table_cap) break;
            bytes += 2 * align256(tb);
        }
    }
    return MINDIST_OK;
}

int prepare_code(const uint64_t *G, int n, int k, uint64_t table_cap, HostCode &hc, uint64_t heavy_cap) {
    hc = HostCode();
    hc.n = n;
    hc.k = k;
    int e = make_plan(G, n, k, hc.P);
    if (e) return e;
    hc.n_gamma = (int)hc.P.sets.size();
    if (hc.n_gamma > kBatchMaxSets) return fail(MINDIST_E_LIMIT, "more than 32 information sets");
    // the kernel's table runs read their binomials from an LDS slice of
    // x < kLdsBinomX (with n <= 512, a code of more rows fits the layout
    // only if every column outside its one information set is zero; the
    // single path runs such codes)
    if (k > kLdsBinomX) return fail(MINDIST_E_LIMIT, "more than 256 rows");
    const Binom &B = BN();
    hc.D.resize(hc.n_gamma);
    hc.dp.resize(hc.n_gamma);
    hc.bcap.resize(hc.n_gamma);
    hc.rows.resize(hc.n_gamma);
    // short codes keep their tables small: their table job would otherwise
    // sit on the launch's critical path (a code's pairs wait for it) and
    // small tables stay in cache while many codes read theirs at once
    const double work = estimated_work(hc);
    if (work < kSmallCodeWork) table_cap = std::min<uint64_t>(table_cap, kSmallCodeTableBytes);
    if (work >= kHeavyCodeWork && heavy_cap) table_cap = std::max<uint64_t>(table_cap, heavy_cap);
    for (int j = 0; j < hc.n_gamma; ++j) {
        const std::vector<int> cols = carried_columns(hc.P, j);
        hc.D[j] = (int)((cols.size() + 31) / 32);
        if (hc.D[j] > kBatchMaxD) return fail(MINDIST_E_LIMIT, "rows wider than 256 bits");
        hc.dp[j] = dp_of_host(hc.D[j]);
        hc.rows[j].assign((size_t)k * hc.dp[j], 0u);
        for (int r = 0; r < k; ++r)
            pack_row(&hc.P.gamma[j][(size_t)r * hc.P.W], cols, &hc.rows[j][(size_t)r * hc.dp[j]], hc.dp[j]);
        int bc = 0;
        for (int b = 1; b <= kBatchMaxB && b <= k; ++b) {
            if (B(k, b) * (uint64_t)hc.dp[j] * 4 > table_cap) break;
            bc = b;
        }
        hc.bcap[j] = bc;
    }
    // the balanced split of the expected top level needs b = top/2; a table
    // is built only if the largest expected pair reads it many times over
    // (C(k,b) at most C(k,top) / kTableReuse): in the persistent kernel an
    // entry costs tens of enumerated codewords to build (a successor step,
    // a scattered store), so a level that is read less pays for itself
    // nowhere near
    const int top = expected_top_level(hc);
    const int want = std::max(1, top / 2);
    for (int &b : hc.bcap) {
        b = std::min(b, want);
        while (b > 1 && B(k, b) > B(k, top) / kTableReuse) --b;
    }
    size_tables(hc);
    return MINDIST_OK;
}

void size_tables(HostCode &hc) {
    // device footprint in three regions: rows (uploaded), right tables (built
    // on the device), witness slots (read back); 256-byte pieces so no cache
    // line is shared between two codes' tables
    const Binom &B = BN();
    const int k = hc.k;
    hc.rows_bytes = hc.tab_bytes = 0;
    for (int j = 0; j < hc.n_gamma; ++j) {
        hc.rows_bytes += align256((size_t)k * hc.dp[j] * 4);
        for (int b = 0; b <= hc.bcap[j]; ++b) hc.tab_bytes += align256(B(k, b) * hc.dp[j] * 4);
        for (int b1 = 1; b1 <= hc.bcap[j]; ++b1) {
            const uint64_t ent = B(k - hc.bcap[j], b1);
            hc.tab_bytes += align256(ent * hc.dp[j] * 4) + align256(ent * 4);
        }
    }
    hc.slot_bytes = align256(sizeof(Slot) * (size_t)(hc.n + 1));
}

void fit_tables(std::vector<HostCode *> &codes, uint64_t budget) {
    uint64_t sum = 0;
    for (HostCode *h : codes) sum += h->tab_bytes;
    while (sum > budget) {
        // the code with the largest tables gives up one level on every set
        HostCode *big = nullptr;
        for (HostCode *h : codes) {
            bool can = false;
            for (int b : h->bcap) can = can || b > 1;
            if (can && (!big || h->tab_bytes > big->tab_bytes)) big = h;
        }
        if (!big) return;
        const uint64_t before = big->tab_bytes;
        for (int &b : big->bcap)
            if (b > 1) --b;
        size_tables(*big);
        sum -= before - big->tab_bytes;
    }
}

void fill_slot(const HostCode &hc, const SlotPlace &pl, unsigned char *rows_stage,
               uint32_t tile_cap, uint64_t seq, BatchCode &bc) {
    std::memset(&bc, 0, sizeof(bc));
    const Binom &B = BN();
    bc.n = hc.n;
    bc.k = hc.k;
    bc.m_full = hc.P.m_full;
    bc.k_m = hc.P.k_m;
    bc.n_gamma = hc.n_gamma;
    bc.W = hc.P.W;
    bc.status = kSlotPending;
    bc.njobs = 0;
    bc.U_found = kInf;
    bc.tile_cap = tile_cap;
    bc.seq = seq;
    uint64_t acc = 0;
    for (int t = 0; t < kBatchTabs; ++t) {
        bc.tab_off[t] = acc;
        const int j = t / kTabsPerSet, r = t % kTabsPerSet;
        if (j >= hc.n_gamma) continue;
        if (r <= kBatchMaxB) {
            if (r <= hc.bcap[j]) acc += B(hc.k, r);
        } else {
            const int b1 = r - (kBatchMaxB + 1);
            if (b1 >= 1 && b1 <= hc.bcap[j]) acc += B(hc.k - hc.bcap[j], b1);
        }
    }
    bc.tab_off[kBatchTabs] = acc;
    size_t ro = 0, to = 0;
    for (int j = 0; j < hc.n_gamma; ++j) {
        BatchSet &s = bc.sets[j];
        s.D = hc.D[j];
        s.dp = hc.dp[j];
        s.stripped = j < hc.P.m_full ? 1 : 0;
        s.bcap = hc.bcap[j];
        const size_t rb = (size_t)hc.k * hc.dp[j] * 4;
        std::memcpy(rows_stage + ro, hc.rows[j].data(), rb);
        s.rows = reinterpret_cast<const uint32_t *>(pl.rows + ro);
        ro += align256(rb);
        for (int b = 0; b <= hc.bcap[j]; ++b) {
            s.rtab[b] = reinterpret_cast<uint32_t *>(pl.tabs + to);
            to += align256(B(hc.k, b) * hc.dp[j] * 4);
        }
        for (int b1 = 1; b1 <= hc.bcap[j]; ++b1) {
            const uint64_t ent = B(hc.k - hc.bcap[j], b1);
            s.otab[b1] = reinterpret_cast<uint32_t *>(pl.tabs + to);
            to += align256(ent * hc.dp[j] * 4);
            s.ocnt[b1] = reinterpret_cast<uint32_t *>(pl.tabs + to);
            to += align256(ent * 4);
        }
    }
    bc.slots = reinterpret_cast<Slot *>(pl.slots);
}

int decode_code(const HostCode &hc, const BatchCode &bc, const unsigned char *arena,
                uint64_t arena_lo, const Slot *slots, mindist_result &out,
                std::vector<mindist_pair> &trace, double wall_hz) {
    std::memset(&out, 0, sizeof(out));
    trace.clear();
    const int n = hc.n, k = hc.k;
    out.n = n;
    out.k = k;
    out.m_full = hc.P.m_full;
    out.k_partial = hc.P.k_m;
    out.n_gamma = hc.n_gamma;
    if (bc.status != kSlotDone) {
        out.d = bc.status < 0 ? bc.status : MINDIST_E_STATE;
        return out.d;
    }
    const Binom &B = BN();
    const uint32_t singleton = (uint32_t)(n - k + 1);
    uint64_t executed = 0, canonical = 0;
    for (int p = 1; p < bc.njobs; ++p) {
        const BatchJob *jb = reinterpret_cast<const BatchJob *>(arena + (size_t)(bc.job[p] - arena_lo) * 128);
        mindist_pair r{};
        r.j = jb->j;
        r.w = jb->w;
        r.L_before = (int)jb->L_before;
        r.L_after = (int)jb->L_after;
        r.U_after = (int)jb->U_after;
        r.pair_min = jb->pair_min == kInf ? -1 : (int)jb->pair_min;
        r.count = jb->count;
        r.executed = jb->executed;
        r.dwords = hc.D[jb->j];
        r.split_a = jb->a;
        r.split_b = jb->b;
        r.split_b2 = jb->b2;
        if (jb->t_open && bc.t_open) {
            const double hz = wall_hz > 0 ? wall_hz : 1e8;
            r.t_start_ms = (double)(jb->t_open - bc.t_open) / hz * 1e3;
            if (jb->t_close >= jb->t_open) r.ms = (double)(jb->t_close - jb->t_open) / hz * 1e3;
        }
        trace.push_back(r);
        executed += r.executed;
        canonical += r.count;
        out.exited_midpair = (jb->exit_flag && jb->executed < jb->count) ? 1 : 0;
    }
    out.pairs_visited = (int)trace.size();
    if (!trace.empty()) {
        out.j_last = trace.back().j;
        out.w_last = trace.back().w;
    }
    out.L_final = (int)bc.L_final;
    out.U_found = bc.U_found == kInf ? n + 1 : (int)bc.U_found;
    out.d = (int)std::min<uint32_t>(bc.U_found, singleton);
    out.executed_total = executed;
    out.canonical_total = canonical;
    {
        // the device sequencer's decisions, rechecked on the host: per-pair
        // bounds, the partial set at every level, mid-pair exit
        CertSpec cs;
        cs.n = n;
        cs.k = k;
        cs.sched = Schedule(k, hc.P.m_full, hc.P.k_m, kPartialAlways);
        std::vector<PairView> views(trace.size());
        for (size_t t = 0; t < trace.size(); ++t) {
            const mindist_pair &r = trace[t];
            views[t] = PairView{r.j, r.w, r.L_before, r.L_after, r.U_after, r.pair_min, r.count, r.executed};
        }
        const int e = certify_trace(cs, views.data(), (int)views.size(), out.d, out.L_final,
                                    out.exited_midpair);
        if (e) return e;
    }
    if (bc.U_found != kInf) {
        const Slot s = slots[bc.U_found];
        if (s.pair < 1 || s.pair >= (uint32_t)bc.njobs)
            return fail(MINDIST_E_CERT, "batch witness slot holds an invalid job index");
        const BatchJob *jb = reinterpret_cast<const BatchJob *>(arena + (size_t)(bc.job[s.pair] - arena_lo) * 128);
        const std::vector<int> rows = witness_rows(k, jb->a, jb->b, jb->b2, s);
        const int e = certify_witness(hc.P, jb->j, rows, jb->w, (int)bc.U_found, out.witness, out.witness_rows);
        if (e) return e;
        out.witness_j = jb->j;
        out.witness_w = jb->w;
    }
    (void)B;
    return MINDIST_OK;
}

// run fn(i) for i in [0, count) on up to `threads` host threads
void parallel_for(int count, int threads, const std::function<void(int)> &fn) {
    threads = std::max(1, std::min(threads, count));
    if (threads == 1) {
        for (int i = 0; i < count; ++i) fn(i);
        return;
    }
    std::atomic<int> next{0};
    std::vector<std::thread> pool;
    for (int t = 0; t < threads; ++t)
        pool.emplace_back([&]() {
            for (int i; (i = next.fetch_add(1)) < count;) fn(i);
        });
    for (auto &th : pool) th.join();
}

int host_threads() {
    const unsigned hw = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(hw ? hw : 1u, 16u));
}

}  // namespace md

using namespace md;

extern "C" int mindist_run_batch(const uint64_t *const *G, const int *n, const int *k, int B,
                                 mindist_result *out, mindist_batch_opts *opts) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!G || !n || !k || !out || B < 1) return fail(MINDIST_E_ARG, "bad batch arguments");
    mindist_batch_opts dflt{};
    mindist_batch_opts &o = opts ? *opts : dflt;
    // right-tile bounds: at least 2048 entries, so a short pair's left tile
    // is one chunk (per-chunk set-up -- claim, left-subset unranking,
    // reductions -- dominated short codes at 256)
    const uint32_t tile_min = o.tile_min > 0 ? (uint32_t)o.tile_min : 2048u;
    const uint32_t tile_max = std::max(tile_min, o.tile_max > 0 ? (uint32_t)o.tile_max : 4096u);
    const int bpc = o.blocks_per_cu > 0 ? o.blocks_per_cu : 4;
    const uint64_t table_cap = (uint64_t)(o.table_kib > 0 ? o.table_kib : 65536) << 10;
    const int jobs_per_code = o.jobs_per_code > 0 ? o.jobs_per_code : 96;
    const bool use_graph = o.use_graph != 0 || opts == nullptr;

    // host preprocessing
    std::vector<HostCode> hc(B);
    std::vector<int> status(B, 0);
    std::vector<std::string> errs(B);
    parallel_for(B, host_threads(), [&](int i) {
        status[i] = prepare_code(G[i], n[i], k[i], table_cap, hc[i], o.table_kib > 0 ? 0 : kHeavyCodeTableBytes);
    });
    const auto t_prep = std::chrono::steady_clock::now();
    // routing: a code expected to enumerate at least 2^direct_log2
    // combinations (or beyond the persistent kernel's limits) runs through
    // the single-code path on a worker thread, where its pairs fill the GPU
    // on their own; the others share the persistent launch, which saves
    // them the per-pair launches and host round trips that dominate short
    // codes
    const bool direct_on = o.direct_log2 >= 0;
    const double direct_min = std::exp2(o.direct_log2 > 0 ? o.direct_log2 : 30);
    std::vector<int> live, direct;
    for (int i = 0; i < B; ++i) {
        if (status[i] == MINDIST_OK && !(direct_on && estimated_work(hc[i]) >= direct_min)) live.push_back(i);
        else if (direct_on && (status[i] == MINDIST_OK || status[i] == MINDIST_E_LIMIT)) direct.push_back(i);
    }
    for (int i = 0; i < B; ++i)
        if (status[i] != MINDIST_OK) {
            std::memset(&out[i], 0, sizeof(out[i]));
            out[i].d = status[i];
            out[i].n = n[i];
            out[i].k = k[i];
        }
    if (live.empty() && direct.empty()) return fail(MINDIST_E_ARG, "no valid code in the batch");
    std::vector<std::vector<mindist_pair>> direct_traces(direct.size());
    double direct_s = 0;
    std::atomic<bool> direct_timed_out{false};
    auto run_direct = [&](double t_offset) -> int {
        // worker threads, each running whole codes through the single path
        // on its own stream; the device runs their kernels side by side
        if (direct.empty()) return MINDIST_OK;
        const auto td = std::chrono::steady_clock::now();
        int dev = 0;
        (void)hipGetDevice(&dev);
        std::atomic<int> next{0};
        std::atomic<int> hard{MINDIST_OK};
        std::string hard_msg;
        std::mutex mu;
        auto worker = [&]() {
            (void)hipSetDevice(dev);
            for (int t; (t = next.fetch_add(1)) < (int)direct.size();) {
                const int i = direct[t];
                mindist_ctx *ctx = nullptr;
                int st = mindist_create(G[i], n[i], k[i], &ctx);
                if (st == MINDIST_OK && o.deadline_s > 0) {
                    const double left = o.deadline_s -
                        std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
                    st = left > 0 ? mindist_set_option(ctx, MINDIST_OPT_DEADLINE_MS, std::max<int64_t>(1, (int64_t)(left * 1e3)))
                                  : MINDIST_E_TIMEOUT;
                }
                if (st == MINDIST_OK) st = mindist_run(ctx, &out[i]);
                if (st == MINDIST_OK) {
                    int np = 0;
                    mindist_get_pairs(ctx, nullptr, 0, &np);
                    direct_traces[t].resize(np);
                    if (np) mindist_get_pairs(ctx, direct_traces[t].data(), np, &np);
                } else {
                    const std::string msg = last_error_text();
                    std::memset(&out[i], 0, sizeof(out[i]));
                    out[i].d = st;
                    out[i].n = n[i];
                    out[i].k = k[i];
                    if (st == MINDIST_E_TIMEOUT) direct_timed_out = true;
                    if (st == MINDIST_E_HIP) {
                        std::lock_guard<std::mutex> lk(mu);
                        hard = st;
                        hard_msg = msg;
                    }
                }
                if (ctx) mindist_destroy(ctx);
                if (o.done_s)
                    o.done_s[i] = t_offset + std::chrono::duration<double>(std::chrono::steady_clock::now() - td).count();
            }
        };
        const int nw = std::min<int>(kBatchDirectWorkers, (int)direct.size());
        std::vector<std::thread> ths;
        for (int w = 1; w < nw; ++w) ths.emplace_back(worker);
        worker();
        for (auto &th : ths) th.join();
        direct_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - td).count();
        if (hard != MINDIST_OK) return fail(hard, hard_msg);
        return MINDIST_OK;
    };
    if (o.done_s)
        for (int i = 0; i < B; ++i) o.done_s[i] = -1.0;
    auto write_pairs = [&](const std::vector<std::vector<mindist_pair>> *persist_traces) {
        if (!o.pairs_index) return;
        int64_t pos = 0;
        std::vector<const std::vector<mindist_pair> *> by_code(B, nullptr);
        if (persist_traces)
            for (size_t s = 0; s < live.size(); ++s) by_code[live[s]] = &(*persist_traces)[s];
        for (size_t t = 0; t < direct.size(); ++t) by_code[direct[t]] = &direct_traces[t];
        for (int i = 0; i < B; ++i) {
            o.pairs_index[i] = pos;
            if (by_code[i])
                for (const auto &r : *by_code[i]) {
                    if (o.pairs && pos < o.pairs_cap) o.pairs[pos] = r;
                    ++pos;
                }
        }
        o.pairs_index[B] = pos;
    };
    if (live.empty()) {
        // every code runs through the single path
        int e = run_direct(0.0);
        if (e) return e;
        uint64_t executed = 0;
        for (int i : direct) if (out[i].d > 0) executed += out[i].executed_total;
        write_pairs(nullptr);
        o.seconds_kernel = direct_s;
        o.wave_s_table = o.wave_s_pair = o.wave_s_flush = 0;
        o.waves = 0;
        o.chunks_table = o.chunks_pair = 0;
        o.seconds_prep = std::chrono::duration<double>(t_prep - t0).count();
        o.executed_total = executed;
        o.seconds_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (direct_timed_out) return fail(MINDIST_E_TIMEOUT, "batch deadline reached before every code finished");
        return MINDIST_OK;
    }
    const int L = (int)live.size();
    {
        // all saved tables of the batch within half of the free device memory
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) {
            std::vector<HostCode *> ptrs;
            for (int i : live) ptrs.push_back(&hc[i]);
            fit_tables(ptrs, free_b / 2);
        }
    }

    // device layout: three regions, each code's pieces at running offsets
    size_t rows_total = 0, tab_total = 0, slot_total = 0;
    std::vector<size_t> ro(L), to(L), so(L);
    int kmax = 1;
    for (int s = 0; s < L; ++s) {
        const HostCode &h = hc[live[s]];
        ro[s] = rows_total;
        to[s] = tab_total;
        so[s] = slot_total;
        rows_total += h.rows_bytes;
        tab_total += h.tab_bytes;
        slot_total += h.slot_bytes;
        kmax = std::max(kmax, h.k);
    }
    const uint64_t arena_units = (uint64_t)L * jobs_per_code * job_bytes(kmax) / 128;
    Engine eng;
    int e = eng.init(L, rows_total, tab_total, slot_total, arena_units, o.stream);
    if (e) return e;
    parallel_for(L, host_threads(), [&](int s) {
        SlotPlace pl{eng.d_rows + ro[s], eng.d_tabs + to[s], eng.d_slots + so[s]};
        fill_slot(hc[live[s]], pl, eng.h_rows + ro[s], tile_max, (uint64_t)s + 1, eng.h_codes[s]);
    });
    const uint32_t quantum = o.chunks_per_visit > 0 ? (uint32_t)o.chunks_per_visit
                             : o.chunks_per_visit < 0 ? 0u : 4u;
    e = eng.run(bpc, tile_min, tile_max, use_graph, o.deadline_s > 0 ? o.deadline_s : 0, quantum);
    if (e) return e;
    e = eng.fetch_all();
    if (e) return e;
    bool timed_out = false;
    for (int s = 0; s < L; ++s)
        if (eng.h_codes[s].status != kSlotDone && eng.h_codes[s].status >= 0) timed_out = true;
    uint64_t executed = 0;
    std::vector<std::vector<mindist_pair>> traces(L);
    std::vector<int> drc(L, 0);
    std::vector<std::string> derr(L);
    parallel_for(L, host_threads(), [&](int s) {
        const int i = live[s];
        const Slot *slots = reinterpret_cast<const Slot *>(eng.h_slots + so[s]);
        drc[s] = decode_code(hc[i], eng.h_codes[s], eng.h_arena, 0, slots, out[i], traces[s], eng.wall_hz);
        if (drc[s]) derr[s] = last_error_text();
    });
    int cert_fail = -1;
    for (int s = 0; s < L; ++s) {
        executed += out[live[s]].executed_total;
        if (drc[s] == MINDIST_E_HIP) return fail(MINDIST_E_HIP, derr[s]);
        if (drc[s] == MINDIST_E_CERT) {
            out[live[s]].d = MINDIST_E_CERT;
            if (cert_fail < 0) cert_fail = s;
        }
    }
    // the codes routed to the single path, after the persistent launch
    e = run_direct(eng.kernel_seconds);
    if (e) return e;
    for (int i : direct) if (out[i].d > 0) executed += out[i].executed_total;
    write_pairs(&traces);
    if (cert_fail >= 0)
        return fail(MINDIST_E_CERT, "batch code " + std::to_string(live[cert_fail]) + ": " + derr[cert_fail]);
    if (timed_out || direct_timed_out)
        return fail(MINDIST_E_TIMEOUT, "batch deadline reached before every code finished");
    o.seconds_kernel = eng.kernel_seconds + direct_s;
    o.wave_s_table = (double)eng.h_g->ticks_table / eng.wall_hz;
    o.wave_s_pair = (double)eng.h_g->ticks_pair / eng.wall_hz;
    o.wave_s_flush = (double)eng.h_g->ticks_flush / eng.wall_hz;
    o.waves = eng.waves;
    o.chunks_table = eng.h_g->chunks_table;
    o.chunks_pair = eng.h_g->chunks_pair;
    if (o.done_s) {
        uint64_t t0 = ~0ull;
        for (int s = 0; s < L; ++s)
            if (eng.h_codes[s].t_open) t0 = std::min<uint64_t>(t0, eng.h_codes[s].t_open);
        for (int s = 0; s < L; ++s) {
            const BatchCode &bc = eng.h_codes[s];
            if (bc.t_done && t0 != ~0ull) o.done_s[live[s]] = (double)(bc.t_done - t0) / eng.wall_hz;
        }
    }
    o.seconds_prep = std::chrono::duration<double>(t_prep - t0).count();
    o.executed_total = executed;
    o.seconds_total = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return MINDIST_OK;
}

// ---------------------------------------------------------------------------
namespace md {

int Engine::init(int slots_, size_t rb, size_t tb, size_t sb, uint64_t au, int64_t user_stream,
                 bool serving) {
    slots = slots_;
    rows_bytes = std::max<size_t>(rb, 256);
    tab_bytes = std::max<size_t>(tb, 256);
    slot_bytes = std::max<size_t>(sb, 256);
    arena_units = std::max<uint64_t>(au, 64);
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(MINDIST_E_HIP, "no HIP device");
    cus = prop.multiProcessorCount;
    d_codes = static_cast<BatchCode *>(dev_alloc(sizeof(BatchCode) * (size_t)slots));
    d_g = static_cast<BatchGlobal *>(dev_alloc(sizeof(BatchGlobal)));
    d_arena = static_cast<unsigned char *>(dev_alloc(arena_units * 128));
    d_rows = static_cast<unsigned char *>(dev_alloc(rows_bytes));
    d_tabs = static_cast<unsigned char *>(dev_alloc(tab_bytes));
    d_slots = static_cast<unsigned char *>(dev_alloc(slot_bytes));
    h_codes = static_cast<BatchCode *>(pinned_alloc(sizeof(BatchCode) * (size_t)slots));
    h_g = static_cast<BatchGlobal *>(pinned_alloc(sizeof(BatchGlobal)));
    h_rows = static_cast<unsigned char *>(pinned_alloc(rows_bytes));
    h_slots = static_cast<unsigned char *>(pinned_alloc(slot_bytes));
    if (!d_codes || !d_g || !d_arena || !d_rows || !d_tabs || !d_slots || !h_codes || !h_g ||
        !h_rows || !h_slots)
        return fail(MINDIST_E_NOMEM, "batch: device or pinned allocation failed");
    if (serving) {
        if (hipHostMalloc((void **)&h_done, sizeof(uint32_t) * (size_t)slots,
                          hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
            hipHostMalloc((void **)&h_stop, 256, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess)
            return fail(MINDIST_E_NOMEM, "server: pinned flag allocation failed");
        std::memset(h_done, 0, sizeof(uint32_t) * (size_t)slots);
        *h_stop = 0;
    }
    if (user_stream) {
        stream = (hipStream_t)user_stream;
        own_stream = false;
    } else {
        stream = stream_get();
        own_stream = true;
    }
    e0 = event_get();
    e1 = event_get();
    if (!stream || !e0 || !e1) return fail(MINDIST_E_HIP, "batch: stream or event creation failed");
    return MINDIST_OK;
}

int Engine::run(int blocks_per_cu, uint32_t tile_min, uint32_t tile_max, bool graph,
                double deadline_s, uint32_t quantum) {
    std::memset(h_g, 0, sizeof(BatchGlobal));
    h_g->arena_cap = arena_units;
    BatchArgs a{};
    a.codes = d_codes;
    a.g = d_g;
    a.arena = d_arena;
    a.binom = device_binom_from(BN().t.data());
    a.n_codes = slots;
    a.serving = 0;
    a.tile_min = tile_min;
    a.tile_max = tile_max;
    a.quantum = quantum;
    {
        int khz = 0;
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
            khz = 100000;
        wall_hz = khz * 1000.0;
        if (deadline_s > 0) a.deadline_ticks = (uint64_t)(deadline_s * wall_hz);
    }
    if (!a.binom) return fail(MINDIST_E_NOMEM, "binomial table upload failed");
    // a persistent grid larger than what is resident would only start its
    // last blocks once the first ones leave
    const int resident = persistent_resident_blocks_per_cu();
    const int blocks = cus * (resident > 0 && blocks_per_cu > resident ? resident : blocks_per_cu);
    waves = blocks * 4;
    auto enqueue = [&]() -> int {
        if (hipMemcpyAsync(d_codes, h_codes, sizeof(BatchCode) * (size_t)slots, hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(d_g, h_g, sizeof(BatchGlobal), hipMemcpyHostToDevice, stream) != hipSuccess ||
            hipMemcpyAsync(d_rows, h_rows, rows_bytes, hipMemcpyHostToDevice, stream) != hipSuccess)
            return fail(MINDIST_E_HIP, "batch: upload failed");
        if (launch_persistent(a, blocks, stream)) return fail(MINDIST_E_HIP, "batch: launch failed");
        return MINDIST_OK;
    };
    if (graph) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(MINDIST_E_HIP, "batch: graph capture failed to start");
        int e = enqueue();
        const hipError_t ec = hipStreamEndCapture(stream, &g);
        if (e) { if (g) (void)hipGraphDestroy(g); return e; }
        if (ec != hipSuccess || hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(MINDIST_E_HIP, "batch: graph capture failed");
        }
        const bool ok = hipEventRecord(e0, stream) == hipSuccess &&
                        hipGraphLaunch(ge, stream) == hipSuccess &&
                        hipEventRecord(e1, stream) == hipSuccess &&
                        hipStreamSynchronize(stream) == hipSuccess;
        (void)hipGraphExecDestroy(ge);
        (void)hipGraphDestroy(g);
        if (!ok) return fail(MINDIST_E_HIP, std::string("batch: graph launch failed: ") +
                                                hipGetErrorString(hipGetLastError()));
    } else {
        if (hipEventRecord(e0, stream) != hipSuccess) return fail(MINDIST_E_HIP, "event record failed");
        int e = enqueue();
        if (e) return e;
        if (hipEventRecord(e1, stream) != hipSuccess || hipStreamSynchronize(stream) != hipSuccess)
            return fail(MINDIST_E_HIP, std::string("batch: kernel failed: ") +
                                           hipGetErrorString(hipGetLastError()));
    }
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    kernel_seconds = ms * 1e-3;
    return MINDIST_OK;
}

int Engine::fetch_all() {
    if (hipMemcpyAsync(h_codes, d_codes, sizeof(BatchCode) * (size_t)slots, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(h_g, d_g, sizeof(BatchGlobal), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(h_slots, d_slots, slot_bytes, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
        return fail(MINDIST_E_HIP, "batch: readback failed");
    // the job records' first lines only (the rest -- chunk counters and
    // groups -- is never read back): ~1/10 of the used arena
    const uint64_t used_units = std::min<uint64_t>(h_g->arena_next, arena_units);
    std::vector<uint32_t> src;
    for (int s = 0; s < slots; ++s) {
        BatchCode &bc = h_codes[s];
        const int nj = std::max(0, std::min<int>(bc.njobs, (int)kBatchMaxPairs));
        for (int p = 0; p < nj; ++p) {
            if (bc.job[p] >= used_units) return fail(MINDIST_E_HIP, "batch: job offset outside the arena");
            src.push_back(bc.job[p]);
            bc.job[p] = (uint32_t)(src.size() - 1);
        }
    }
    const uint32_t n = (uint32_t)src.size();
    pinned_free(h_lines);
    h_lines = static_cast<unsigned char *>(pinned_alloc((size_t)std::max<uint32_t>(n, 1) * 128));
    uint32_t *d_src = static_cast<uint32_t *>(dev_alloc((size_t)std::max<uint32_t>(n, 1) * 4));
    unsigned char *d_lines = static_cast<unsigned char *>(dev_alloc((size_t)std::max<uint32_t>(n, 1) * 128));
    int rc = MINDIST_OK;
    if (!h_lines || !d_src || !d_lines) rc = fail(MINDIST_E_NOMEM, "batch: readback buffers");
    if (rc == MINDIST_OK && n &&
        (hipMemcpyAsync(d_src, src.data(), (size_t)n * 4, hipMemcpyHostToDevice, stream) != hipSuccess ||
         launch_gather_lines(d_arena, d_src, n, d_lines, stream) != 0 ||
         hipMemcpyAsync(h_lines, d_lines, (size_t)n * 128, hipMemcpyDeviceToHost, stream) != hipSuccess ||
         hipStreamSynchronize(stream) != hipSuccess))
        rc = fail(MINDIST_E_HIP, "batch: job readback failed");
    (void)hipStreamSynchronize(stream);
    dev_free(d_src);
    dev_free(d_lines);
    h_arena = h_lines;
    return rc;
}

Engine::~Engine() {
    if (stream) (void)hipStreamSynchronize(stream);
    dev_free(d_codes);
    dev_free(d_g);
    dev_free(d_arena);
    dev_free(d_rows);
    dev_free(d_tabs);
    dev_free(d_slots);
    pinned_free(h_codes);
    pinned_free(h_g);
    pinned_free(h_rows);
    pinned_free(h_slots);
    pinned_free(h_lines);
    if (h_done) (void)hipHostFree(h_done);
    if (h_stop) (void)hipHostFree(h_stop);
    event_put(e0);
    event_put(e1);
    if (own_stream) stream_put(stream);
}

}  // namespace md
