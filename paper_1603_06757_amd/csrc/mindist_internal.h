// mindist_internal.h -- data shared by the host scheduler and the HIP kernels.
//
// Enumeration scheme (the GPU form of Section 3.4, saved additions): a pair
// (Gamma_j, w) covers every w-subset of the k rows.  A w-subset is split as
// X u Y with |X| = a, |Y| = b = w - a and max X < min Y.  X ("left") is
// produced per lane: its colexicographic rank rho is unranked and its a rows
// are added once per chunk.  Y ("right") comes from a saved table of all
// b-subset sums, read by the whole wave at the same index (scalar loads), so
// each codeword costs one row addition plus the weight.  The table is stored
// so that the right subsets allowed after a left subset with maximum e, i.e.
// the b-subsets of [e+1, k), are its first C(k-1-e, b) entries: entry i is
// the b-subset {k-1-z : z in colex_unrank_b(i)}.  This is the lexicographic
// table of Section 3.4 read from its end, so the paper's right restriction
// C(k,b) - C(k-e-1,b) becomes the prefix length C(k-e-1,b).
//
// Left subsets in colex order are grouped by their maximum e, and the right
// ranges of larger e are prefixes of those of smaller e, so a wave whose 64*B
// items straddle several e runs one loop and masks lanes past their range.
#pragma once
#include <stddef.h>
#include <stdint.h>

#if defined(__HIPCC__)
#define MD_HD __host__ __device__
#else
#define MD_HD
#endif

namespace md {

constexpr int kBinomT = 65;          // binomial table: t in [0, 64]
constexpr int kBinomX = 513;         // x in [0, 512]
constexpr uint32_t kInf = 0xFFFFFFFFu;

// one group of left tiles whose first item has maximum element e
struct GroupEntry {
    uint64_t chunk_base;   // first chunk id of the group
    uint64_t lt_begin;     // first left tile
    uint64_t n_rt;         // right tiles per left tile
    uint32_t nr_first;     // C(k-1-e, b): right entries of the tile's first item
    uint32_t e;
};

struct PairStat {
    uint32_t pair_min;     // least weight over the pair (kInf if none yet)
    uint32_t pad;
    uint64_t executed;     // combinations evaluated
    uint64_t wsum;         // sum of weights (verify mode)
    uint64_t pad2;
};

struct Slot {              // witness of weight v: written once, by the wave
    uint32_t pair;         // whose atomicMin moved U_found down to v
    uint32_t i;            // right table index
    uint64_t rho;          // colex rank of the left subset
};

struct DevState {
    uint32_t U_found;      // least weight found so far in the run (kInf = none)
    uint32_t exit_flag;    // set when U_found <= the bound before the pair
    uint32_t cancelled;
    uint32_t pad;
    uint64_t claimed;      // chunks claimed in the run (for cancel_after)
    uint64_t pad2;
    // followed by Slot slots[513], PairStat pairs[max_pairs] and the chunk
    // dispensers: kCounters counters per pair, each on its own 128-byte line
};

constexpr int kCounters = 8;         // interleaved chunk dispensers per pair
constexpr int kCounterStride = 16;   // uint64 words between two counters (128 B)

MD_HD inline size_t state_bytes(int max_pairs) {
    return sizeof(DevState) + sizeof(Slot) * 513 + sizeof(PairStat) * (size_t)max_pairs +
           sizeof(uint64_t) * kCounters * kCounterStride * (size_t)max_pairs;
}
MD_HD inline Slot *state_slots(DevState *s) { return reinterpret_cast<Slot *>(s + 1); }
MD_HD inline PairStat *state_pairs(DevState *s) {
    return reinterpret_cast<PairStat *>(reinterpret_cast<Slot *>(s + 1) + 513);
}
// counter q of pair p
MD_HD inline uint64_t *state_counter(DevState *s, int max_pairs, int p, int q) {
    uint64_t *base = reinterpret_cast<uint64_t *>(state_pairs(s) + max_pairs);
    return base + ((size_t)p * kCounters + q) * kCounterStride;
}

struct PairArgs {
    const uint32_t *rows;      // k rows x dp words (stripped or full)
    const uint32_t *table;     // right table: C(k,b) entries x dp words
    const uint32_t *ltable;    // left table: entry rho = rows of colex_unrank_a(rho)
                               // (nullptr: lanes unrank and add the rows themselves)
    const uint64_t *binom;     // kBinomX x kBinomT
    const GroupEntry *groups;  // left-tile-major chunk order (order = 0)
    const uint64_t *rprefix;   // right-tile-major order (order = 1): chunk ids
                               // of right tile r start at rprefix[r]
    DevState *st;
    uint64_t n_items;          // C(k-b, a): left subsets that have a right partner
    uint64_t total_chunks;
    uint64_t cancel_after;     // 0 = off
    int32_t ngroups, k, a, b;
    uint32_t T;                // right tile length
    uint32_t offset;           // added to every weight (w for identity-stripped rows)
    uint32_t L_prev;           // bound before the pair (exit threshold)
    uint32_t pair;             // index into the pair statistics
    uint32_t midpair_exit;
    int32_t max_pairs;         // layout of the state block
    uint32_t order;            // 0: chunk = (left tile, right tile) left-major, 1: right-major
    uint32_t n_rt;             // right tiles (order = 1)
    uint32_t counters;         // chunk dispensers in use (1 or kCounters)
    uint32_t pad;
};

struct TableArgs {
    const uint32_t *rows;
    const uint64_t *binom;
    uint32_t *table;
    uint64_t entries;
    int32_t k, b, dp;
    int32_t reflect;           // 1: right table (rows k-1-z), 0: left table (rows z)
};

// kernel launchers (mindist_kernels.hip)
int launch_init_state(DevState *st, int max_pairs, void *stream);
int launch_build_table(const TableArgs &ta, int D, void *stream);
// items: lane items per chunk (2 or 4)
int launch_enum_pair(const PairArgs &pa, int D, int items, int verify, int blocks, void *stream);
int max_dwords();
int launch_peak(const uint32_t *tab, uint32_t steps, uint32_t *out, int D, int blocks, void *stream);

}  // namespace md
