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
    uint64_t next_chunk;   // chunk dispenser
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
    // followed by Slot slots[513] and PairStat pairs[max_pairs]
};

MD_HD inline size_t state_bytes(int max_pairs) {
    return sizeof(DevState) + sizeof(Slot) * 513 + sizeof(PairStat) * (size_t)max_pairs;
}
MD_HD inline Slot *state_slots(DevState *s) { return reinterpret_cast<Slot *>(s + 1); }
MD_HD inline PairStat *state_pairs(DevState *s) {
    return reinterpret_cast<PairStat *>(reinterpret_cast<Slot *>(s + 1) + 513);
}

struct PairArgs {
    const uint32_t *rows;      // k rows x dp words (stripped or full)
    const uint32_t *table;     // right table: C(k,b) entries x dp words
    const uint64_t *binom;     // kBinomX x kBinomT
    const GroupEntry *groups;
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
    uint32_t pad;
};

struct TableArgs {
    const uint32_t *rows;
    const uint64_t *binom;
    uint32_t *table;
    uint64_t entries;
    int32_t k, b, dp;
};

// kernel launchers (mindist_kernels.hip)
int launch_init_state(DevState *st, int max_pairs, void *stream);
int launch_build_table(const TableArgs &ta, int D, void *stream);
int launch_enum_pair(const PairArgs &pa, int D, int verify, int blocks, void *stream);
int max_dwords();

}  // namespace md
