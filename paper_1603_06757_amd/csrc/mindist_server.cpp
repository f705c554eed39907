// mindist_server.cpp -- continuous batching of arriving codes on one GPU.
//
// Two engines serve the same queue.
//
// Engine 0 (default): worker threads, each taking the next waiting code and
// running the single-code path on it (context, pair launches with the next
// pairs queued ahead, mailbox reads) on its own stream.  The device runs the
// kernels of the codes in flight side by side: short pairs of one code fill
// the compute units another code's short pairs leave idle, and a code's
// latency is that of the single-code path.
//
// Engine 1: the persistent multi-code kernel keeps every resident code
// moving (pair after pair, Algorithm 1's control on the device); codes
// expected to enumerate at least 2^route_log2 combinations (and codes beyond
// the kernel's layout) run through the single-code path on 4 worker threads
// beside it instead, the kernel then holding 2 blocks per CU so that their
// kernels find room: alone in the persistent kernel such a code's pairs run
// on the few waves their chunks occupy, several times slower.  A code
// that arrives while it runs is admitted into it: the manager thread writes
// the code's descriptor and packed rows into the slot's inbox entry in
// pinned host memory and publishes the slot in a ring; one of the kernel's
// polling waves copies it to the device and makes the slot pending, and the
// waves take it up like any other (tables are built on the device by each
// code's first job).  A slot and a pool range serve at most one code per
// launch -- a wave may still touch a finished code's records for a moment
// -- so freed ones return at the next launch.  The manager stops the launch
// ("an epoch") only when a waiting code cannot be admitted into it but would
// be after a relaunch (every free slot already used in this launch, pool
// ranges waiting to return, rows too large for an inbox entry), when no code
// is left, or after 10 s.  Waves finish the chunk they hold and add it to
// its job before leaving, so a stopped code resumes exactly where it was in
// the next launch; codes admitted between launches are written by plain
// copies.  While a launch runs, a finished code's last wave copies what the
// host needs (descriptor, job records, witness slot) into pinned host memory
// and then sets the code's completion word there; the manager decodes it
// without stopping the others and without any device copy.
//
// Device memory: slot descriptors and per-slot job arena segments are sized
// at creation; rows, saved tables and witness slots of each code come from
// one pool allocated at creation and handed out first-fit, so admission
// never allocates device memory while the kernel runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/mindist.h"
#include "mindist_batch.h"
#include "mindist_batch_engine.h"
#include "mindist_plan.h"
#include "mindist_pool.h"

namespace md {
namespace {

constexpr size_t kAlign = 256;
constexpr int kRouteWorkers = 4;     // engine 1: single-path workers for the routed codes
constexpr double kRouteLaunchMax = 0.02;   // s: longest launch while routed codes are in flight

size_t round_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// first-fit allocator over [0, size) with coalescing of freed ranges
class RangePool {
public:
    explicit RangePool(size_t size = 0) { if (size) free_[0] = size; }
    bool alloc(size_t n, size_t &off) {
        n = round_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            off = it->first;
            const size_t rest = it->second - n;
            free_.erase(it);
            if (rest) free_[off + n] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = round_up(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
private:
    std::map<size_t, size_t> free_;
};

struct Request {
    uint64_t tag = 0;
    HostCode hc;                 // engine 1
    std::vector<uint64_t> G;     // engine 0: the caller's matrix
    int n = 0, k = 0;
    double t_submit = 0, t_admit = 0;
    size_t bytes = 0;            // rows + tables + witness slots
};

struct Resident {
    std::unique_ptr<Request> req;
    size_t off = 0;              // in the device pool
    uint64_t seq = 0;
    bool fresh = false;          // admitted, not yet written to the device
    bool used = false;           // held a code during the current launch
};

}  // namespace
}  // namespace md

struct mindist_server {
    mindist_server_opts o{};
    int device = 0;
    int cus = 256;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;
    std::condition_variable cv;       // submits, completions, shutdown
    std::deque<std::unique_ptr<md::Request>> pending;
    std::deque<std::unique_ptr<md::Request>> routed;   // engine 1: codes for the single-path workers
    int routed_active = 0;                  // engine 1: routed codes being run
    double route_min = 0;                   // engine 1: estimated combinations from which a code is routed (0: none)
    std::deque<std::unique_ptr<mindist_server_result>> done;
    std::vector<md::Resident> slots;
    int resident = 0;
    bool quit = false;
    mindist_server_stats st{};

    // device state
    md::BatchCode *d_codes = nullptr;
    md::BatchGlobal *d_g = nullptr;
    unsigned char *d_arena = nullptr;
    unsigned char *d_pool = nullptr;
    md::BatchCode *h_codes = nullptr;       // pinned staging of descriptors
    md::BatchGlobal *h_g = nullptr;
    uint32_t *h_done = nullptr, *h_stop = nullptr;   // pinned, coherent
    uint32_t *dv_done = nullptr, *dv_stop = nullptr; // their device addresses
    md::ServeMirror *h_mirror = nullptr, *dv_mirror = nullptr;   // finished codes' records
    md::ServeInbox *h_inbox = nullptr, *dv_inbox = nullptr;      // codes admitted during a launch
    uint32_t *h_ring = nullptr, *dv_ring = nullptr;              // their slots, in order
    uint32_t *h_admit = nullptr, *dv_admit = nullptr;            // [0]: ring count, [32]: copied
    uint32_t published = 0;                 // ring entries of the current launch
    bool running = false;                   // a launch is in flight (manager thread)
    std::vector<std::pair<size_t, size_t>> retired;   // pool ranges freed during the launch
    hipStream_t stream = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    uint64_t seg_units = 0;                 // job arena units per slot
    md::RangePool pool;
    uint64_t next_seq = 1;
    double wall_hz = 1e8;                   // device wall-clock rate
    std::thread mgr;
    std::vector<std::thread> workers;       // engine 0
    size_t bytes_budget = 0, bytes_in_flight = 0;   // engine 0: device footprint admission
    std::string fatal;                      // first device error seen by the manager

    double clock() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace md {
namespace {

// Decode the finished code in slot s from the mirror the kernel wrote to
// pinned host memory; frees its slot and pool range.  Called by the manager
// thread while the kernel may still be running (no device copy involved).
void collect(mindist_server *S, int s, std::vector<unsigned char> &arena_host,
             std::vector<Slot> &slot_host) {
    Resident &r = S->slots[s];
    HostCode &hc = r.req->hc;
    auto res = std::make_unique<mindist_server_result>();
    std::memset(res.get(), 0, sizeof(*res));
    res->tag = r.req->tag;
    res->t_submit = r.req->t_submit;
    res->t_admit = r.req->t_admit;
    const ServeMirror &m = S->h_mirror[s];
    BatchCode bc;
    std::memset(&bc, 0, sizeof(bc));
    std::memcpy(&bc, m.code, kMirrorCodeBytes);
    // job p's first line sits at m.jobs[p]
    const int nj = std::max(0, std::min<int>(bc.njobs, kBatchMaxPairs));
    arena_host.assign((size_t)std::max(nj, 1) * 128, 0);
    for (int p = 0; p < nj; ++p) {
        std::memcpy(arena_host.data() + (size_t)p * 128, m.jobs[p], 128);
        bc.job[p] = (uint32_t)p;
    }
    slot_host.assign((size_t)hc.n + 1, Slot{});
    if (bc.U_found != kInf && bc.U_found <= (uint32_t)hc.n) slot_host[bc.U_found] = m.witness;
    std::vector<mindist_pair> trace;
    int status = decode_code(hc, bc, arena_host.data(), 0, slot_host.data(), res->result, trace,
                             S->wall_hz);
    res->n_pairs = (int)std::min<size_t>(trace.size(), MINDIST_SERVER_MAX_PAIRS);
    for (int t = 0; t < res->n_pairs; ++t) res->pairs[t] = trace[t];
    res->status = status;
    if (status != MINDIST_OK && res->result.d >= 0) res->result.d = status;
    res->t_done = S->clock();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->running) S->retired.emplace_back(r.off, r.req->bytes);   // returns at the next launch
    else S->pool.release(r.off, r.req->bytes);
    r.req.reset();
    r.fresh = false;
    --S->resident;
    ++S->st.completed;
    S->done.push_back(std::move(res));
    S->cv.notify_all();
}

// Move waiting requests that fit into free slots (submission order among
// those that fit).  Caller holds the lock.
int admit_locked(mindist_server *S) {
    int admitted = 0;
    for (auto it = S->pending.begin(); it != S->pending.end();) {
        int free_slot = -1;
        for (int s = 0; s < (int)S->slots.size(); ++s)
            if (!S->slots[s].req) { free_slot = s; break; }
        if (free_slot < 0) break;
        size_t off = 0;
        if (!S->pool.alloc((*it)->bytes, off)) { ++it; continue; }
        Resident &r = S->slots[free_slot];
        r.req = std::move(*it);
        r.req->t_admit = S->clock();
        r.off = off;
        r.seq = S->next_seq++;
        r.fresh = true;
        r.used = true;
        ++S->resident;
        ++S->st.admitted;
        ++admitted;
        it = S->pending.erase(it);
    }
    return admitted;
}

// While a launch runs: move waiting requests that fit into slots not used
// in this launch (submission order among those that fit; rows within an
// inbox entry).  Returns the slots.  Caller holds the lock.
std::vector<int> admit_live_locked(mindist_server *S) {
    std::vector<int> out;
    int s_next = 0;
    for (auto it = S->pending.begin(); it != S->pending.end();) {
        if ((*it)->hc.rows_bytes > kInboxRowsBytes) { ++it; continue; }
        while (s_next < (int)S->slots.size() && (S->slots[s_next].req || S->slots[s_next].used)) ++s_next;
        if (s_next >= (int)S->slots.size()) break;
        size_t off = 0;
        if (!S->pool.alloc((*it)->bytes, off)) { ++it; continue; }
        Resident &r = S->slots[s_next];
        r.req = std::move(*it);
        r.req->t_admit = S->clock();
        r.off = off;
        r.seq = S->next_seq++;
        r.fresh = false;
        r.used = true;
        ++S->resident;
        ++S->st.admitted;
        ++S->st.admitted_live;
        out.push_back(s_next);
        it = S->pending.erase(it);
    }
    return out;
}

// Write slot s's code into its inbox entry and publish it to the running
// kernel (the ring entry, then the count, released).
void publish_live(mindist_server *S, int s, uint32_t tile_max) {
    Resident &r = S->slots[s];
    HostCode &hc = r.req->hc;
    ServeInbox &in = S->h_inbox[s];
    unsigned char *base = S->d_pool + r.off;
    SlotPlace pl{base, base + round_up(hc.rows_bytes), base + round_up(hc.rows_bytes) + round_up(hc.tab_bytes)};
    fill_slot(hc, pl, in.rows, tile_max, r.seq, in.code);
    in.code.arena_lo = (uint64_t)s * S->seg_units;
    in.code.arena_hi = (uint64_t)(s + 1) * S->seg_units;
    in.code.arena_next = in.code.arena_lo;
    in.rows_dst = (uint64_t)(uintptr_t)pl.rows;
    in.rows_bytes = (uint32_t)hc.rows_bytes;
    __atomic_store_n(&S->h_done[s], 0u, __ATOMIC_RELAXED);
    S->h_ring[S->published] = (uint32_t)s;
    ++S->published;
    __atomic_store_n(&S->h_admit[0], S->published, __ATOMIC_RELEASE);
}

// Write the freshly admitted slots to the device (the kernel is stopped).
int upload_fresh(mindist_server *S, const uint32_t tile_max) {
    std::vector<std::vector<unsigned char>> stage;
    for (int s = 0; s < (int)S->slots.size(); ++s) {
        Resident &r = S->slots[s];
        if (!r.req || !r.fresh) continue;
        HostCode &hc = r.req->hc;
        unsigned char *base = S->d_pool + r.off;
        SlotPlace pl{base, base + round_up(hc.rows_bytes), base + round_up(hc.rows_bytes) + round_up(hc.tab_bytes)};
        stage.emplace_back(round_up(hc.rows_bytes));
        fill_slot(hc, pl, stage.back().data(), tile_max, r.seq, S->h_codes[s]);
        S->h_codes[s].arena_lo = (uint64_t)s * S->seg_units;
        S->h_codes[s].arena_hi = (uint64_t)(s + 1) * S->seg_units;
        S->h_codes[s].arena_next = S->h_codes[s].arena_lo;
        S->h_done[s] = 0;
        if (hipMemcpyAsync(S->d_codes + s, S->h_codes + s, sizeof(BatchCode), hipMemcpyHostToDevice, S->stream) != hipSuccess ||
            hipMemcpyAsync(pl.rows, stage.back().data(), hc.rows_bytes, hipMemcpyHostToDevice, S->stream) != hipSuccess)
            return fail(MINDIST_E_HIP, "server: slot upload failed");
        r.fresh = false;
    }
    if (hipStreamSynchronize(S->stream) != hipSuccess) return fail(MINDIST_E_HIP, "server: slot upload failed");
    return MINDIST_OK;
}

void manager(mindist_server *S) {
    (void)hipSetDevice(S->device);
    const uint32_t tile_min = 2048, tile_max = 4096;   // as the batch defaults
    // with codes routed to single-path workers, 1 block per CU (half of each
    // SIMD's registers) leaves room for their kernels beside the persistent
    // one; otherwise as many as fit (2)
    const int bpc_req = S->o.blocks_per_cu > 0 ? S->o.blocks_per_cu : S->route_min > 0 ? 1 : 4;
    const int resident_bpc = persistent_resident_blocks_per_cu();
    const int blocks = S->cus * (resident_bpc > 0 && bpc_req > resident_bpc ? resident_bpc : bpc_req);
    const double epoch_min = (S->o.epoch_min_ms > 0 ? S->o.epoch_min_ms : 0.5) * 1e-3;
    // a launch with no code left waits this long for the next arrivals
    // (admitted into it) before it ends
    const double linger = S->o.linger_ms > 0 ? S->o.linger_ms * 1e-3 : S->o.linger_ms < 0 ? 0.0 : 0.2;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, S->device) != hipSuccess || khz <= 0)
        khz = 100000;
    S->wall_hz = khz * 1000.0;
    std::vector<unsigned char> arena_host;
    std::vector<Slot> slot_host;
    auto die = [&](const std::string &msg) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->fatal = msg;
        S->quit = true;
        S->cv.notify_all();
    };
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(S->mu);
            // between launches: ranges freed during the last one return to
            // the pool, and a slot is used only if it holds a code
            for (auto &rg : S->retired) S->pool.release(rg.first, rg.second);
            S->retired.clear();
            for (auto &r : S->slots) r.used = (bool)r.req;
            admit_locked(S);
            if (S->resident == 0) {
                if (S->quit) return;
                S->cv.wait(lk, [&] { return S->quit || !S->pending.empty(); });
                continue;
            }
        }
        if (upload_fresh(S, tile_max)) {
            die(last_error_text());
            return;
        }
        // one launch
        std::memset(S->h_g, 0, sizeof(BatchGlobal));
        {
            // the codes this launch starts with: the pair planner gives each
            // its share of the waves (the kernel counts the ones admitted later)
            std::lock_guard<std::mutex> lk(S->mu);
            S->h_g->live0 = (uint32_t)std::max(1, S->resident);
            S->running = true;
        }
        S->published = 0;
        __atomic_store_n(&S->h_admit[0], 0u, __ATOMIC_RELAXED);
        __atomic_store_n(&S->h_admit[32], 0u, __ATOMIC_RELAXED);
        *reinterpret_cast<volatile uint32_t *>(S->h_stop) = 0;
        std::atomic_thread_fence(std::memory_order_seq_cst);
        BatchArgs a{};
        a.codes = S->d_codes;
        a.g = S->d_g;
        a.arena = S->d_arena;
        a.binom = device_binom_from(BN().t.data());
        a.host_done = S->dv_done;
        a.host_stop = S->dv_stop;
        a.mirror = S->dv_mirror;
        a.inbox = S->dv_inbox;
        a.admit_ring = S->dv_ring;
        a.admit_count = S->dv_admit;
        a.admit_ack = S->dv_admit + 32;
        a.n_codes = (int)S->slots.size();
        a.serving = 1;
        a.tile_min = tile_min;
        a.tile_max = tile_max;
        a.deadline_ticks = (uint64_t)(10.0 * khz * 1000.0);   // a launch never outlives 10 s
        a.quantum = S->o.chunks_per_visit > 0 ? (uint32_t)S->o.chunks_per_visit
                    : S->o.chunks_per_visit < 0 ? 0u : 4u;
        if (!a.binom ||
            hipMemcpyAsync(S->d_g, S->h_g, sizeof(BatchGlobal), hipMemcpyHostToDevice, S->stream) != hipSuccess ||
            hipEventRecord(S->ev0, S->stream) != hipSuccess || launch_persistent(a, blocks, S->stream) ||
            hipEventRecord(S->ev1, S->stream) != hipSuccess) {
            die("server: launch failed");
            return;
        }
        const double t_launch = S->clock();
        double t_idle = -1;                 // when the launch last became empty
        bool stop_sent = false;
        for (;;) {
            const hipError_t q = hipEventQuery(S->ev1);
            // completions announced by the kernel
            for (int s = 0; s < (int)S->slots.size(); ++s) {
                Resident &r = S->slots[s];
                if (!r.req || r.fresh) continue;
                const uint32_t v = __atomic_load_n(&S->h_done[s], __ATOMIC_ACQUIRE);
                if (v == (uint32_t)r.seq) collect(S, s, arena_host, slot_host);
            }
            if (q != hipErrorNotReady) break;
            // codes that arrived: into the running kernel
            std::vector<int> live;
            if (!stop_sent) {
                std::lock_guard<std::mutex> lk(S->mu);
                if (!S->quit) live = admit_live_locked(S);
            }
            for (int s : live) publish_live(S, s, tile_max);
            bool stop = false;
            {
                std::unique_lock<std::mutex> lk(S->mu);
                const double now = S->clock();
                if (S->resident > 0) t_idle = -1;
                else if (t_idle < 0) t_idle = now;
                // Streams beyond the process's hardware queues share them, and
                // a queue runs its kernels in order: a routed code's kernels
                // may wait behind the persistent launch.  While routed codes
                // are in flight, a launch neither lingers nor runs longer
                // than kRouteLaunchMax (then it is relaunched over its codes)
                const bool routed_busy = S->routed_active > 0 || !S->routed.empty();
                if (S->quit) stop = true;
                else if (S->resident == 0 && S->pending.empty() && now - t_idle >= (routed_busy ? 0.0 : linger))
                    stop = true;
                else if (routed_busy && now - t_launch >= kRouteLaunchMax) stop = true;
                else if (!S->pending.empty() && now - t_launch >= epoch_min) {
                    // a waiting code could not come in: stop only if a relaunch
                    // would let it (a free slot used earlier in this launch,
                    // pool ranges waiting to return, rows beyond an inbox entry)
                    bool free_slot = false;
                    for (auto &r : S->slots) free_slot = free_slot || !r.req;
                    bool wide = false;
                    for (auto &p : S->pending) wide = wide || p->hc.rows_bytes > kInboxRowsBytes;
                    stop = free_slot && (!S->retired.empty() || wide ||
                                         std::none_of(S->slots.begin(), S->slots.end(),
                                                      [](const Resident &r) { return !r.req && !r.used; }));
                }
                if (!stop && live.empty()) S->cv.wait_for(lk, std::chrono::microseconds(50));
            }
            if (stop && !stop_sent) {
                __atomic_store_n(S->h_stop, 1u, __ATOMIC_RELEASE);
                stop_sent = true;
            }
        }
        if (hipStreamSynchronize(S->stream) != hipSuccess) {
            die(std::string("server: kernel failed: ") + hipGetErrorString(hipGetLastError()));
            return;
        }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, S->ev0, S->ev1);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            ++S->st.epochs;
            S->st.seconds_kernel += ms * 1e-3;
            S->running = false;
            // published codes the kernel did not copy in before it ended are
            // written by the next launch's upload
            const uint32_t copied = __atomic_load_n(&S->h_admit[32], __ATOMIC_ACQUIRE);
            for (uint32_t i = copied; i < S->published; ++i) S->slots[S->h_ring[i]].fresh = true;
        }
        // codes that finished right before the launch ended
        for (int s = 0; s < (int)S->slots.size(); ++s) {
            Resident &r = S->slots[s];
            if (!r.req || r.fresh) continue;
            if (__atomic_load_n(&S->h_done[s], __ATOMIC_ACQUIRE) == (uint32_t)r.seq)
                collect(S, s, arena_host, slot_host);
        }
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->quit) return;
    }
}

// Engine 0: one worker thread.  A code is admitted when a worker is free
// and its device footprint fits beside the codes in flight (submission
// order among the codes that fit); the single-code path allocates nothing
// per code after warm-up (process-wide caches of device memory, streams
// and events).
//
// routed (engine 1): the same, over the codes routed to the single path by
// their estimated work, beside the persistent kernel; no memory budget (the
// single path's own device memory), one code per worker.
void direct_worker(mindist_server *S, bool routed) {
    (void)hipSetDevice(S->device);
    const int table_mib = S->o.table_kib > 0 && !routed ? std::max(1, S->o.table_kib / 1024) : 0;
    auto &queue = routed ? S->routed : S->pending;
    for (;;) {
        std::unique_ptr<Request> req;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            auto fitting = queue.end();
            S->cv.wait(lk, [&] {
                if (S->quit) return true;
                fitting = std::find_if(queue.begin(), queue.end(), [&](const auto &r) {
                    return routed || S->bytes_in_flight + r->bytes <= S->bytes_budget;
                });
                return fitting != queue.end();
            });
            if (S->quit) return;
            req = std::move(*fitting);
            queue.erase(fitting);
            req->t_admit = S->clock();
            if (routed) {
                ++S->routed_active;
                ++S->st.routed;
            } else {
                S->bytes_in_flight += req->bytes;
                ++S->resident;
            }
            ++S->st.admitted;
        }
        auto res = std::make_unique<mindist_server_result>();
        std::memset(res.get(), 0, sizeof(*res));
        res->tag = req->tag;
        res->t_submit = req->t_submit;
        res->t_admit = req->t_admit;
        mindist_ctx *ctx = nullptr;
        int status = mindist_create(req->G.data(), req->n, req->k, &ctx);
        if (status == MINDIST_OK && table_mib) status = mindist_set_option(ctx, MINDIST_OPT_TABLE_MIB, table_mib);
        if (status == MINDIST_OK) status = mindist_run(ctx, &res->result);
        double kernel_s = 0;
        if (ctx) {
            int np = 0;
            if (status == MINDIST_OK &&
                mindist_get_pairs(ctx, res->pairs, MINDIST_SERVER_MAX_PAIRS, &np) == MINDIST_OK)
                res->n_pairs = std::min(np, MINDIST_SERVER_MAX_PAIRS);
            for (int t = 0; t < res->n_pairs; ++t) kernel_s += res->pairs[t].dev_ms * 1e-3;
            mindist_destroy(ctx);
        }
        res->status = status;
        if (status != MINDIST_OK && res->result.d >= 0) res->result.d = status;
        res->t_done = S->clock();
        std::lock_guard<std::mutex> lk(S->mu);
        if (routed) {
            --S->routed_active;
        } else {
            --S->resident;
            S->bytes_in_flight -= req->bytes;
        }
        ++S->st.completed;
        S->st.seconds_kernel += kernel_s;
        S->done.push_back(std::move(res));
        S->cv.notify_all();
    }
}

void release(mindist_server *S) {
    if (S->stream) (void)hipStreamSynchronize(S->stream);
    dev_free(S->d_codes);
    dev_free(S->d_g);
    dev_free(S->d_arena);
    dev_free(S->d_pool);
    pinned_free(S->h_codes);
    pinned_free(S->h_g);
    if (S->h_done) (void)hipHostFree(S->h_done);
    if (S->h_stop) (void)hipHostFree(S->h_stop);
    if (S->h_mirror) (void)hipHostFree(S->h_mirror);
    if (S->h_inbox) (void)hipHostFree(S->h_inbox);
    if (S->h_ring) (void)hipHostFree(S->h_ring);
    if (S->h_admit) (void)hipHostFree(S->h_admit);
    if (S->stream) stream_put(S->stream);
    if (S->ev0) event_put(S->ev0);
    if (S->ev1) event_put(S->ev1);
}

}  // namespace
}  // namespace md

using namespace md;

extern "C" int mindist_server_create(const mindist_server_opts *opts, mindist_server **out) {
    if (!out) return fail(MINDIST_E_ARG, "null output pointer");
    *out = nullptr;
    auto S = std::make_unique<mindist_server>();
    if (opts) S->o = *opts;
    if (S->o.engine != 0 && S->o.engine != 1) return fail(MINDIST_E_ARG, "engine must be 0 or 1");
    if (S->o.engine == 0) {
        const int workers = S->o.max_active > 0 ? S->o.max_active : 8;
        if (workers > 256) return fail(MINDIST_E_ARG, "max_active too large for engine 0 (at most 256 workers)");
        if (hipGetDevice(&S->device) != hipSuccess) return fail(MINDIST_E_HIP, "no HIP device");
        // warm the process-wide caches the first codes would otherwise pay
        // for: one stream per worker, the binomial table
        {
            std::vector<hipStream_t> ss;
            for (int t = 0; t < workers; ++t) ss.push_back(stream_get());
            for (hipStream_t st : ss)
                if (st) stream_put(st);
            if (!device_binom_from(BN().t.data())) return fail(MINDIST_E_NOMEM, "binomial table upload failed");
        }
        S->bytes_budget = S->o.device_bytes > 0 ? (size_t)S->o.device_bytes : (size_t)8 << 30;
        S->t0 = std::chrono::steady_clock::now();
        mindist_server *raw = S.get();
        for (int t = 0; t < workers; ++t) raw->workers.emplace_back(direct_worker, raw, false);
        *out = S.release();
        return MINDIST_OK;
    }
    const int slots = S->o.max_active > 0 ? S->o.max_active : 256;
    if (slots > 65536) return fail(MINDIST_E_ARG, "max_active too large");
    const size_t pool_bytes = S->o.device_bytes > 0 ? (size_t)S->o.device_bytes : (size_t)8 << 30;
    const int jobs = S->o.jobs_per_code > 0 ? S->o.jobs_per_code : 96;
    hipDeviceProp_t prop;
    if (hipGetDevice(&S->device) != hipSuccess || hipGetDeviceProperties(&prop, S->device) != hipSuccess)
        return fail(MINDIST_E_HIP, "no HIP device");
    S->cus = prop.multiProcessorCount;
    S->t0 = std::chrono::steady_clock::now();
    S->slots.resize(slots);
    S->seg_units = (uint64_t)jobs * job_bytes(MINDIST_MAX_N / 2) / 128;
    S->d_codes = static_cast<BatchCode *>(dev_alloc(sizeof(BatchCode) * (size_t)slots));
    S->d_g = static_cast<BatchGlobal *>(dev_alloc(sizeof(BatchGlobal)));
    S->d_arena = static_cast<unsigned char *>(dev_alloc(S->seg_units * 128 * (size_t)slots));
    S->d_pool = static_cast<unsigned char *>(dev_alloc(pool_bytes));
    S->h_codes = static_cast<BatchCode *>(pinned_alloc(sizeof(BatchCode) * (size_t)slots));
    S->h_g = static_cast<BatchGlobal *>(pinned_alloc(sizeof(BatchGlobal)));
    if (!S->d_codes || !S->d_g || !S->d_arena || !S->d_pool || !S->h_codes || !S->h_g) {
        release(S.get());
        return fail(MINDIST_E_NOMEM, "server: device or pinned allocation failed");
    }
    if (hipHostMalloc((void **)&S->h_done, sizeof(uint32_t) * (size_t)slots,
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
        hipHostMalloc((void **)&S->h_stop, 256, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void **)&S->dv_done, S->h_done, 0) != hipSuccess ||
        hipHostGetDevicePointer((void **)&S->dv_stop, S->h_stop, 0) != hipSuccess ||
        hipHostMalloc((void **)&S->h_mirror, sizeof(ServeMirror) * (size_t)slots,
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void **)&S->dv_mirror, S->h_mirror, 0) != hipSuccess ||
        hipHostMalloc((void **)&S->h_inbox, sizeof(ServeInbox) * (size_t)slots,
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void **)&S->dv_inbox, S->h_inbox, 0) != hipSuccess ||
        hipHostMalloc((void **)&S->h_ring, sizeof(uint32_t) * (size_t)slots,
                      hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void **)&S->dv_ring, S->h_ring, 0) != hipSuccess ||
        hipHostMalloc((void **)&S->h_admit, 256, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer((void **)&S->dv_admit, S->h_admit, 0) != hipSuccess) {
        release(S.get());
        return fail(MINDIST_E_NOMEM, "server: pinned flag allocation failed");
    }
    std::memset(S->h_ring, 0xFF, sizeof(uint32_t) * (size_t)slots);
    std::memset(S->h_admit, 0, 256);
    std::memset(S->h_done, 0, sizeof(uint32_t) * (size_t)slots);
    *S->h_stop = 0;
    // every slot starts empty on the device
    std::memset(S->h_codes, 0, sizeof(BatchCode) * (size_t)slots);
    for (int s = 0; s < slots; ++s) S->h_codes[s].status = kSlotEmpty;
    S->stream = stream_get();
    S->ev0 = event_get();
    S->ev1 = event_get();
    if (!S->stream || !S->ev0 || !S->ev1 ||
        hipMemcpyAsync(S->d_codes, S->h_codes, sizeof(BatchCode) * (size_t)slots, hipMemcpyHostToDevice,
                       S->stream) != hipSuccess ||
        hipStreamSynchronize(S->stream) != hipSuccess) {
        release(S.get());
        return fail(MINDIST_E_HIP, "server: stream setup failed");
    }
    S->pool = RangePool(pool_bytes);
    if (S->o.route_log2 >= 0) {
        S->route_min = std::ldexp(1.0, S->o.route_log2 > 0 ? S->o.route_log2 : 24);
        // warm one stream per routed worker and the binomial table
        std::vector<hipStream_t> ss;
        for (int t = 0; t < kRouteWorkers; ++t) ss.push_back(stream_get());
        for (hipStream_t st : ss)
            if (st) stream_put(st);
        if (!device_binom_from(BN().t.data())) {
            release(S.get());
            return fail(MINDIST_E_NOMEM, "binomial table upload failed");
        }
    }
    mindist_server *raw = S.get();
    raw->mgr = std::thread(manager, raw);
    if (raw->route_min > 0)
        for (int t = 0; t < kRouteWorkers; ++t) raw->workers.emplace_back(direct_worker, raw, true);
    *out = S.release();
    return MINDIST_OK;
}

extern "C" int mindist_server_submit(mindist_server *S, const uint64_t *G, int n, int k, uint64_t tag) {
    if (!S || !G) return fail(MINDIST_E_ARG, "null argument");
    auto r = std::make_unique<Request>();
    r->tag = tag;
    r->t_submit = S->clock();
    if (S->o.engine == 0) {
        // validate and size here (the caller learns of a bad matrix at
        // once); the worker plans again inside mindist_create.  Footprint:
        // rows, right and left saved tables up to the levels the estimated
        // distance needs (within the table cap), and the run's state.
        const uint64_t table_cap = S->o.table_kib > 0 ? (uint64_t)S->o.table_kib << 10 : kTableCapDefault;
        int e = single_path_bytes(G, n, k, table_cap, r->bytes);
        if (e) return e;
        if (r->bytes > S->bytes_budget) return fail(MINDIST_E_NOMEM, "code does not fit the server's device memory");
        r->n = n;
        r->k = k;
        r->G.assign(G, G + (size_t)k * ((n + 63) / 64));
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->quit) return fail(MINDIST_E_STATE, "server is shutting down");
        S->pending.push_back(std::move(r));
        ++S->st.submitted;
        S->cv.notify_all();
        return MINDIST_OK;
    }
    const uint64_t table_cap = (uint64_t)(S->o.table_kib > 0 ? S->o.table_kib : 65536) << 10;
    int e = prepare_code(G, n, k, table_cap, r->hc);
    if (e == MINDIST_E_LIMIT && S->route_min > 0) {
        // beyond the persistent kernel's layout: the single path runs it
        r->n = n;
        r->k = k;
        r->G.assign(G, G + (size_t)k * ((n + 63) / 64));
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->quit) return fail(MINDIST_E_STATE, "server is shutting down");
        S->routed.push_back(std::move(r));
        ++S->st.submitted;
        S->cv.notify_all();
        return MINDIST_OK;
    }
    if (e) return e;
    if (S->route_min > 0 && estimated_work(r->hc) >= S->route_min) {
        r->n = n;
        r->k = k;
        r->G.assign(G, G + (size_t)k * ((n + 63) / 64));
        r->hc = HostCode();
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->quit) return fail(MINDIST_E_STATE, "server is shutting down");
        S->routed.push_back(std::move(r));
        ++S->st.submitted;
        S->cv.notify_all();
        return MINDIST_OK;
    }
    const size_t pool_bytes = S->o.device_bytes > 0 ? (size_t)S->o.device_bytes : (size_t)8 << 30;
    // one code may take at most a quarter of the pool: lower its table levels if needed
    std::vector<HostCode *> one{&r->hc};
    fit_tables(one, pool_bytes / 4);
    r->bytes = round_up(r->hc.rows_bytes) + round_up(r->hc.tab_bytes) + round_up(r->hc.slot_bytes);
    if (r->bytes > pool_bytes) return fail(MINDIST_E_NOMEM, "code does not fit the server's device memory");
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->quit) return fail(MINDIST_E_STATE, S->fatal.empty() ? "server is shutting down" : S->fatal);
    S->pending.push_back(std::move(r));
    ++S->st.submitted;
    S->cv.notify_all();
    return MINDIST_OK;
}

extern "C" int mindist_server_poll(mindist_server *S, mindist_server_result *out, int cap, int *n_out) {
    if (!S || !n_out || (cap > 0 && !out)) return fail(MINDIST_E_ARG, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    int n = 0;
    while (n < cap && !S->done.empty()) {
        out[n++] = *S->done.front();
        S->done.pop_front();
    }
    *n_out = n;
    if (n == 0 && S->quit && !S->fatal.empty()) return fail(MINDIST_E_HIP, S->fatal);
    return MINDIST_OK;
}

extern "C" int mindist_server_wait(mindist_server *S, double timeout_s) {
    if (!S) return fail(MINDIST_E_ARG, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    const auto until = std::chrono::steady_clock::now() +
                       std::chrono::microseconds((int64_t)(std::max(timeout_s, 0.0) * 1e6));
    const bool ok = S->cv.wait_until(lk, until, [&] {
        return S->quit || (S->pending.empty() && S->resident == 0 && S->routed.empty() &&
                           S->routed_active == 0);
    });
    if (!S->fatal.empty()) return fail(MINDIST_E_HIP, S->fatal);
    return ok ? MINDIST_OK : fail(MINDIST_E_TIMEOUT, "server: codes still waiting or running");
}

extern "C" double mindist_server_clock(const mindist_server *S) { return S ? S->clock() : 0.0; }

extern "C" int mindist_server_stats_get(const mindist_server *S, mindist_server_stats *out) {
    if (!S || !out) return fail(MINDIST_E_ARG, "null argument");
    auto *M = const_cast<mindist_server *>(S);
    std::lock_guard<std::mutex> lk(M->mu);
    *out = M->st;
    out->resident = M->resident + M->routed_active;
    out->pending = (int32_t)(M->pending.size() + M->routed.size());
    return MINDIST_OK;
}

extern "C" void mindist_server_destroy(mindist_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->quit = true;
        S->cv.notify_all();
    }
    if (S->h_stop) __atomic_store_n(S->h_stop, 1u, __ATOMIC_RELEASE);
    if (S->mgr.joinable()) S->mgr.join();
    for (auto &t : S->workers)
        if (t.joinable()) t.join();   // a code being run finishes first
    release(S);
    delete S;
}
