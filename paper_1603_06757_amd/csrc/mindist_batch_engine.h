// mindist_batch_engine.h -- host-side pieces of the persistent multi-code
// path, shared by mindist_run_batch and the server.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <string>
#include <vector>

#include "../../include/mindist.h"
#include "mindist_batch.h"
#include "mindist_plan.h"

namespace md {

const char *last_error_text();

// one code prepared on the host
struct HostCode {
    int n = 0, k = 0, n_gamma = 0;
    Plan P;
    std::vector<int> D, dp, bcap;               // per set
    std::vector<std::vector<uint32_t>> rows;    // per set, k x dp packed words
    size_t rows_bytes = 0, tab_bytes = 0, slot_bytes = 0;
};

// where a slot's pieces live on the device
struct SlotPlace {
    unsigned char *rows, *tabs, *slots;
};

// heavy_cap: per-table cap for codes expected at or above kHeavyCodeWork
// combinations (0 = the same cap for every code)
int prepare_code(const uint64_t *G, int n, int k, uint64_t table_cap, HostCode &hc, uint64_t heavy_cap = 0);
// validate G and estimate the device bytes the single-code path holds for
// it (rows, saved right and left tables up to half the expected top level,
// rounded up, within the table cap; run state)
int single_path_bytes(const uint64_t *G, int n, int k, uint64_t table_cap, size_t &bytes);
// device bytes of a prepared code from its per-set table levels (bcap)
void size_tables(HostCode &hc);
// lower the table levels of the codes with the largest tables until all
// tables together fit in `budget` bytes (or every set is down to one level)
void fit_tables(std::vector<HostCode *> &codes, uint64_t budget);
void fill_slot(const HostCode &hc, const SlotPlace &pl, unsigned char *rows_stage,
               uint32_t tile_cap, uint64_t seq, BatchCode &bc);
// arena: host copy of the job arena from unit arena_lo on
int decode_code(const HostCode &hc, const BatchCode &bc, const unsigned char *arena,
                uint64_t arena_lo, const Slot *slots, mindist_result &out,
                std::vector<mindist_pair> &trace, double wall_hz = 1e8);
size_t job_bytes(int k);
void parallel_for(int count, int threads, const std::function<void(int)> &fn);
int host_threads();
// combinations Algorithm 1 is expected to enumerate for a prepared code (every
// pair while the bound is below a Gilbert-Varshamov estimate of d)
double estimated_work(const HostCode &hc);

// device buffers and launch of the persistent kernel over `slots` codes
struct Engine {
    int slots = 0;
    int cus = 256;
    BatchCode *d_codes = nullptr;
    BatchGlobal *d_g = nullptr;
    unsigned char *d_arena = nullptr, *d_rows = nullptr, *d_tabs = nullptr, *d_slots = nullptr;
    size_t rows_bytes = 0, tab_bytes = 0, slot_bytes = 0;
    uint64_t arena_units = 0;
    BatchCode *h_codes = nullptr;       // pinned mirrors
    BatchGlobal *h_g = nullptr;
    unsigned char *h_rows = nullptr, *h_slots = nullptr, *h_arena = nullptr;
    uint32_t *h_done = nullptr, *h_stop = nullptr;   // serving: host-visible flags
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double kernel_seconds = 0;
    double wall_hz = 1e8;               // device wall-clock rate
    int waves = 0;                      // waves of the last launch
    unsigned char *h_lines = nullptr;   // pinned: first line of every job, gathered

    int init(int slots, size_t rows_bytes, size_t tab_bytes, size_t slot_bytes,
             uint64_t arena_units, int64_t user_stream, bool serving = false);
    // upload every slot descriptor, the rows and the global state; launch the
    // persistent kernel (inside one captured hipGraph when graph is set) and
    // wait for it
    int run(int blocks_per_cu, uint32_t tile_min, uint32_t tile_max, bool graph,
            double deadline_s = 0, uint32_t quantum = 4);
    // read back the descriptors, the slots and the first line of every job
    // the codes opened (gathered on the device into one dense array; each
    // code's job offsets are rewritten to indices into it, so h_arena reads
    // like the arena with 128-byte lines)
    int fetch_all();
    ~Engine();
};

}  // namespace md
