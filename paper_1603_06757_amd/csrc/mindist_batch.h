// mindist_batch.h -- the device-side scheduler shared by mindist_run_batch and
// the server: many codes in one persistent launch.
//
// Every code slot goes through
//   PENDING -> (a wave opens the table job) -> TABLES -> pair 1 -> pair 2 ... -> DONE
// on the device.  A "job" is a record with a chunk dispenser (claim), a
// completion counter (done) and the number of chunks that will complete
// (expected).  Waves pick a code, claim a chunk of its open job, run it, and
// the wave that completes a job's last chunk opens the code's next job: the
// next pair of Algorithm 1 in canonical order (w ascending, j ascending,
// partial set last), or DONE once L >= U.  The job records live in an arena
// and are never reused within a launch, so a wave that claims on a job that
// has closed simply gets an index past its end.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include "mindist_internal.h"

namespace md {

constexpr int kBatchMaxSets = 32;     // information sets per code
constexpr int kBatchMaxB = 6;         // right tables b = 0..6 per set
constexpr int kBatchMaxPairs = 256;   // jobs per code (table job + pairs)
constexpr int kBatchMaxD = 8;         // 32-bit words carried per row (n <= 256)
// left subsets per lane: 4 up to 4 words per codeword (the matrix-core
// inner loop then multiplies each 32-entry block of right sums by 8 column
// tiles; on the vector ALUs each scalar table line serves 256 codewords of
// the wave), 2 above (the vector-ALU loop holds 4 x D words of left sums
// without spilling only up to D = 4)
constexpr int kBatchItemsMaxD4 = 4;
constexpr int kBatchItemsWide = 2;
// product chains per wave of the matrix-core loop (pairs of up to 4 words):
// two would keep more of the loop's values in scratch beside the
// scheduler's state
constexpr int kBatchMfmaChains = 1;
MD_HD constexpr int batch_items(int D) { return D <= 4 ? kBatchItemsMaxD4 : kBatchItemsWide; }
constexpr int kTableChunk = 4096;     // table entries per table-job chunk (at most)
constexpr int kTableChunkMin = 256, kTableChunksWanted = 16;
// LDS words per wave for the rows of the set a table chunk builds (k rows
// of dp words; a set that does not fit is read from global memory) or the
// chunk groups of the pair it works on, and the block's slice of the
// binomial table, C(x, t) for x < 256 and t <= 8, from which lanes unrank
// their left subsets (subsets of up to 8 rows): 4 waves x 4 KB + 18 KB per
// block, 34 KB (the kernel's registers hold 2 blocks per CU)
constexpr int kRowsLds = 1024;
constexpr int kLdsBinomX = 256, kLdsBinomT = 9;
// a saved table of C(k,b) entries is built only if C(k,b) <= C(k,top) /
// kTableReuse, top = the expected last level of the code
constexpr uint64_t kTableReuse = 1024;
// codes expected to enumerate fewer combinations than this keep every
// saved table within kSmallCodeTableBytes
constexpr double kSmallCodeWork = 536870912.0;         // 2^29
constexpr uint64_t kSmallCodeTableBytes = 256u << 10;  // 256 KiB
// codes expected to enumerate at least 2^34 combinations may keep tables up
// to the single path's cap (with the default per-table cap): their large
// pairs then take the same balanced split, whose right runs are longer
constexpr double kHeavyCodeWork = 17179869184.0;       // 2^34
constexpr uint64_t kHeavyCodeTableBytes = 1ull << 30;  // 1 GiB
// tables of set j: right tables b = 0..bcap (shift 0) at t = j*kTabsPerSet + b,
// outer tables b1 = 1..bcap over rows [0, k-bcap) (shift bcap, with inner
// counts) at t = j*kTabsPerSet + (kBatchMaxB+1) + b1
constexpr int kTabsPerSet = 2 * (kBatchMaxB + 1);
constexpr int kBatchTabs = kBatchMaxSets * kTabsPerSet;

enum : int32_t {
    kSlotActive = 0,
    kSlotDone = 1,
    kSlotPending = 2,
    kSlotOpening = 3,
    kSlotEmpty = 4,
    // negative values: MINDIST_E_* errors
};

struct BatchSet {
    const uint32_t *rows;                  // k x dp
    uint32_t *rtab[kBatchMaxB + 1];        // right tables b = 0..bcap (built on device)
    uint32_t *otab[kBatchMaxB + 1];        // outer tables b1 = 1..bcap, shift bcap
    uint32_t *ocnt[kBatchMaxB + 1];        // their inner counts
    int32_t D, dp, stripped, bcap;
};

constexpr int kJobCounters = 8;       // chunk dispensers per job (one cache line each)
constexpr uint64_t kQuantumJobChunks = 1024;   // jobs this large ignore the chunks-per-visit quantum
// waves that take part in a job: kPickersPerChunk per chunk, at least
// kPickersMin (the rest pass it over without touching it); with at most
// kFewLiveCodes codes live, the Few figures
constexpr uint64_t kPickersPerChunk = 4, kPickersMin = 256;
constexpr uint64_t kPickersPerChunkFew = 1, kPickersMinFew = 64;
constexpr uint32_t kFewLiveCodes = 4;
constexpr int kBatchDirectWorkers = 8;   // threads running a batch's codes routed to the single path

// one job of a code; GroupEntry groups[ngroups] follow the struct.
// Chunks are handed out by nctr counters: counter r hands out chunks
// r, r + nctr, r + 2*nctr, ...; a wave starts at its home counter and moves
// on when that one is drained, so claims spread over nctr cache lines.
// Waves count their completed chunks (and fold their pair minimum and
// evaluated combinations) privately and add them to `done` once, when they
// find the job drained.
struct alignas(128) BatchJob {
    int32_t kind;                 // 0 = table job, 1 = enumeration pair
    int32_t j, w, a, b;
    uint32_t T;                   // pair: right tile length; table job: entries per chunk
    uint32_t L_before, offset, ngroups;
    int32_t b2;                   // inner subset size (0: two-level split)
    uint64_t n_items, total_chunks, count;
    uint32_t pair_min, exit_flag, L_after, U_after;
    uint64_t executed;
    uint64_t expected;            // chunks that complete before the job closes
    uint32_t nctr, pad_a;         // counters in use (1..kJobCounters)
    uint64_t t_open, t_close;     // device wall clock: job opened, last chunk counted
    uint64_t pad_b[2];
    alignas(128) uint64_t done;   // completed chunks
    uint32_t drained_mask;        // bit r: counter r found past its end (shared, so that a
                                  // wave leaving a job need not try every counter)
    uint32_t pad_e;
    uint64_t pad_d[14];
    struct alignas(128) Counter {
        uint64_t v;
        uint64_t pad[15];
    } claim[kJobCounters];
};

// A slot's descriptor.  The first 128-byte line holds only what waves read
// and write with device-scope atomics while a launch runs (every wave
// looking for work reads it); the rest is written once, before the status
// leaves kSlotEmpty, and read with plain loads.  A descriptor is a whole
// number of lines, so that no line of a slot admitted while a launch runs
// can already sit in some XCD's L2 (slots are not reused within a launch).
struct alignas(128) BatchCode {
    int32_t status;               // kSlot* or a negative error
    int32_t njobs;                // jobs opened (the open one is njobs-1)
    int32_t drained;              // njobs value whose open job was found fully
                                  // claimed (a hint for waves looking for work)
    uint32_t U_found;             // least weight found (kInf = none)
    uint32_t line0_pad[28];
    int32_t n, k, m_full, k_m, n_gamma, W;
    uint32_t tile_cap;            // largest right tile for this code
    uint32_t L_final, U_final;
    uint64_t seq;                 // submission sequence number (server)
    uint64_t t_open, t_done;      // device wall clock: table job opened, code finished
    // serving: the code's own job arena segment [arena_lo, arena_hi) and its
    // next free unit (the batch path allocates from BatchGlobal::arena_next)
    uint64_t arena_lo, arena_hi, arena_next;
    uint32_t job[kBatchMaxPairs]; // arena offsets (128-byte units) of the jobs
    Slot *slots;                  // n+1 witness slots
    uint64_t tab_off[kBatchTabs + 1];   // table entries before table t (t = j*(B+1)+b)
    BatchSet sets[kBatchMaxSets];
};

// Serving: what a finished code leaves in pinned host memory for the host
// to decode while the kernel keeps running -- its descriptor up to the job
// offsets, the first cache line of each job record (every field the host
// reads lives there) and the witness slot at its least weight.
constexpr size_t kMirrorCodeBytes = offsetof(BatchCode, slots);
struct ServeMirror {
    unsigned char code[(kMirrorCodeBytes + 15) / 16 * 16];
    unsigned char jobs[kBatchMaxPairs][128];
    Slot witness;
};

// Serving: a code the host admits while the launch runs -- its descriptor
// and packed rows, in pinned host memory, copied to the device by a polling
// wave (rows to rows_dst, a device address in the code's pool range).
constexpr size_t kInboxRowsBytes = 32u << 10;
struct ServeInbox {
    BatchCode code;
    uint64_t rows_dst;
    uint32_t rows_bytes, pad;
    unsigned char rows[kInboxRowsBytes];
};

struct BatchGlobal {
    uint32_t codes_done;          // batch: codes finished (done or error)
    uint32_t stop;                // serving: the host's stop request, mirrored on the device
    uint64_t arena_next;          // 128-byte units handed out
    uint64_t arena_cap;
    // profile (summed over waves at exit): wall-clock ticks spent in table
    // chunks, in enumeration chunks, in flushes (with the job control they
    // run); chunks of each kind
    uint64_t ticks_table, ticks_pair, ticks_flush;
    uint64_t chunks_table, chunks_pair;
    uint32_t live0;               // codes to run when the launch starts (0: every slot), plus
                                  // those admitted since
    uint32_t admit_done;          // serving: ring entries copied to the device this launch
    uint32_t admit_lock;          // serving: held by the wave copying them
    uint64_t pad1[7];
};

struct BatchArgs {
    BatchCode *codes;
    BatchGlobal *g;
    unsigned char *arena;
    const uint64_t *binom;
    uint32_t *host_done;          // serving: per slot completion word in pinned host memory
    ServeMirror *mirror;          // serving: per slot result mirror in pinned host memory
    const uint32_t *host_stop;    // serving: set by the host to end the launch
    // serving: codes admitted while the launch runs (pinned host memory):
    // inbox entries per slot, the ring of their slot indices (n_codes
    // entries), its count (written by the host) and the count copied so far
    // (written back by the device); null: no admission during the launch
    const ServeInbox *inbox;
    const uint32_t *admit_ring;
    const uint32_t *admit_count;
    uint32_t *admit_ack;
    int32_t n_codes;              // code slots
    int32_t serving;              // 0: end when every code is done; 1: end on host_stop
    uint32_t tile_min;            // right tile length bounds
    uint32_t tile_max;
    uint64_t deadline_ticks;      // wall-clock ticks after which every wave leaves (0 = none)
    uint32_t quantum;             // chunks a wave runs on one job per visit (0 = until drained)
    uint32_t pad_q;
};

int launch_persistent(const BatchArgs &a, int blocks, void *stream);
// copy the 128-byte arena lines src[0..n) (arena offsets in 128-byte units)
// to dst[0..n): the first line of each job record holds every field the
// host decodes
int launch_gather_lines(const unsigned char *arena, const uint32_t *src, uint32_t n, unsigned char *dst,
                        void *stream);
// blocks of 256 threads of the persistent kernel that fit on one CU at once
// (0 if the runtime cannot tell)
int persistent_resident_blocks_per_cu();

}  // namespace md
