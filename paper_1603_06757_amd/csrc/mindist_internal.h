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
//
// Three-level split (large w with small saved tables): X u Y1 u Y2 with
// |X| = a per lane, Y1 a b1-subset of rows (max X, k-b2) from the outer
// table (uniform loop) and Y2 a b2-subset of rows (max Y1, k) from the inner
// table (uniform inner loop over its first C(k-1-max Y1, b2) entries).  The
// inner loop is the two-level hot loop with the lane sums L ^ Y1 held fixed,
// so a lane subset covers C(k-1-e, b1+b2) codewords instead of C(k-1-e, b).
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
constexpr int kMfmaMaxD = 4;         // words per codeword the matrix-core inner loop takes
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
static_assert(sizeof(GroupEntry) == 32, "group entries are copied as four 64-bit words");

// One wave's totals over the chunks it ran in a pair, written with plain
// stores when the wave ends (no atomics on a shared line at the end of a
// launch, when every wave finishes at about the same moment).
struct WavePart {
    uint32_t pair_min;     // least weight (kInf if none)
    uint32_t pad;
    uint64_t executed;     // combinations evaluated
    uint64_t wsum;         // sum of weights (verify mode)
    uint64_t t0, t1;       // device wall clock when the wave started and ended
};

struct Slot {              // witness of weight v: written once, by the wave
    uint32_t pair;         // whose atomicMin moved U_found down to v
    uint32_t i;            // right (outer) table index
    uint32_t i2;           // inner table index (three-level split only)
    uint32_t pad;
    uint64_t rho;          // colex rank of the left subset
    uint64_t pad2;
};

// What the publishing kernel behind a pair's launch leaves in pinned host
// memory: the run state, the pair's statistics reduced over its waves and
// the witness slot of the current U_found, published by seq = pair + 1 once
// the rest is written (the host waits on seq instead of synchronising and
// copying back).  Pair p uses mailbox p % kMailRing, so kMailRing - 1 pairs
// can be launched ahead of the one being read.
struct PairMail {
    uint32_t seq;
    uint32_t U_found;
    uint32_t exit_flag;
    uint32_t cancelled;
    uint32_t pair_min;
    uint32_t pad;
    uint64_t executed;
    uint64_t wsum;
    uint64_t t_begin, t_end;   // device wall clock: first wave start, last wave end
    uint64_t pad2;
    Slot witness;          // slot[U_found] (unset while U_found = kInf)
};
constexpr int kMailRing = 16;
constexpr int kGroupMax = 8;          // pairs of one launch at most
constexpr uint32_t kMaxSlot = 512;    // witness slots 0..kMaxSlot, one per weight (n <= 512)


struct DevState {
    uint32_t U_found;      // least weight found so far in the run (kInf = none)
    uint32_t exit_flag;    // set when U_found <= the bound before the pair
    uint32_t cancelled;
    uint32_t U_base;       // U_found after the previous launch (its publish kernel
                           // writes it; kInf before the first)
    uint64_t claimed;      // chunks claimed in the run (for cancel_after)
    uint64_t pad2;
    // followed by Slot slots[kMaxSlot + 1], the chunk dispensers (kCounters
    // counters per pair, each on its own 128-byte line) and, per pair, the
    // least weight found by that pair and the pairs before it in its launch
};

constexpr int kCounters = 8;         // interleaved chunk dispensers per pair
constexpr int kCounterStride = 16;   // uint64 words between two counters (128 B)

MD_HD inline size_t state_bytes(int max_pairs) {
    return sizeof(DevState) + sizeof(Slot) * (kMaxSlot + 1) +
           sizeof(uint64_t) * kCounters * kCounterStride * (size_t)max_pairs +
           sizeof(uint32_t) * (size_t)max_pairs;
}
MD_HD inline Slot *state_slots(DevState *s) { return reinterpret_cast<Slot *>(s + 1); }
// counter q of pair p
MD_HD inline uint64_t *state_counter(DevState *s, int max_pairs, int p, int q) {
    (void)max_pairs;
    uint64_t *base = reinterpret_cast<uint64_t *>(state_slots(s) + kMaxSlot + 1);
    return base + ((size_t)p * kCounters + q) * kCounterStride;
}
// least weight found by pair p and the pairs before it in its launch
MD_HD inline uint32_t *state_prefix_min(DevState *s, int max_pairs) {
    return reinterpret_cast<uint32_t *>(state_counter(s, max_pairs, max_pairs, 0));
}

struct PairArgs {
    const uint32_t *rows;      // k rows x dp words (stripped or full)
    const uint32_t *table;     // right table: C(k,b) entries x dp words
    const uint32_t *ltable;    // left table: entry rho = rows of colex_unrank_a(rho)
                               // (nullptr: lanes unrank and add the rows themselves)
    const uint32_t *table2;    // three-level split: inner right table (b2-subsets)
    const uint32_t *cnt2;      // three-level split: inner entries of each outer entry
    const uint64_t *binom;     // kBinomX x kBinomT
    const GroupEntry *groups;  // left-tile-major chunk order (order = 0)
    const uint64_t *rprefix;   // right-tile-major order (order = 1): chunk ids
                               // of right tile r start at rprefix[r]
    DevState *st;
    uint64_t n_items;          // C(k-b, a): left subsets that have a right partner
    uint64_t total_chunks;
    uint64_t cancel_after;     // 0 = off
    int32_t ngroups, k, a, b;
    int32_t b2;                // 0: two-level split (left | right), else inner size
    uint32_t T;                // right tile length
    uint32_t offset;           // added to every weight (w for identity-stripped rows)
    uint32_t L_prev;           // bound before the pair (exit threshold)
    uint32_t pair;             // index into the pair statistics
    uint32_t midpair_exit;
    int32_t max_pairs;         // layout of the state block
    uint32_t order;            // 0: chunk = (left tile, right tile) left-major, 1: right-major
    uint32_t n_rt;             // right tiles (order = 1)
    uint32_t counters;         // chunk dispensers in use (1 or kCounters)
    uint32_t waves;            // waves of this launch (grid blocks x 4); wave v
                               // runs chunk v first, the dispensers hand out
                               // chunks waves, waves + 1, ...
    WavePart *parts;           // waves entries: each wave's totals
};

// One launch: up to kGroupMax consecutive pairs of Algorithm 1, pair g on
// blocks [block_start[g], block_start[g+1]) (its own chunks, counters,
// per-wave totals and mailbox).  Pair g is cut once the least weight of the
// previous launches (U_base) or of pairs 0..g of this launch reaches its
// bound: Algorithm 1 would then stop at or before pair g, so the pairs it
// visits are enumerated exactly as one launch per pair would.
struct GroupArgs {
    PairArgs p[kGroupMax];
    uint32_t block_start[kGroupMax + 1];
    uint32_t n;                // pairs in this launch
};

// Saved sums of r-subsets: entry i is the sum of the rows of colex_unrank_r(i)
// (left table, reflect = 0) or of the rows {k-1-shift-z} (right tables,
// reflect = 1; shift = b2 > 0 builds the outer table of a three-level split
// over rows [0, k-b2), with cnt2[i] = C(b2 + min z, b2) inner entries).
struct TableArgs {
    const uint32_t *rows;
    const uint64_t *binom;
    uint32_t *table;
    uint32_t *cnt2;            // outer tables only (else nullptr)
    uint64_t entries;
    int32_t k, b, dp;
    int32_t reflect;
    int32_t shift;
    // the same kind of table one level down (shift 0, b >= 2), or nullptr.
    // In colex order the b-subsets with largest element m are the entries
    // [C(m,b), C(m+1,b)), and entry C(m,b) + r is {m} with the (b-1)-subset
    // of rank r (r < C(m,b-1)), so entry C(m,b) + r = row(m) + prev[r]
    // (row k-1-m for the reflected right tables)
    const uint32_t *prev;
};

// kernel launchers (mindist_kernels.hip)
int launch_init_state(DevState *st, int max_pairs, void *stream);
int launch_build_table(const TableArgs &ta, int D, void *stream);
// items: lane items per chunk (2 or 4)
// all pairs of one launch share D and the lane items
// mfma: the two-level pairs of at most kMfmaMaxD words run their full
// 32-entry blocks on the int8 matrix cores (ignored with verify)
int launch_enum_pair(const GroupArgs &ga, int D, int items, int verify, int mfma, void *stream);
// workgroups of 256 threads of the matrix-core enumeration kernel (D words,
// items lane items) one CU holds at once; 0 if the runtime cannot tell
int enum_mfma_resident_blocks(int D, int items);
// one block: reduce the waves' totals of every pair of the launch, read the
// run state and publish them to the pairs' mailboxes (mail[pair %
// kMailRing]), then record U_found as the next launch's U_base (launched
// right behind the enumeration kernel)
int launch_publish_pair(const GroupArgs &ga, PairMail *mail, void *stream);
int max_dwords();
// p[0..count) = v (a fill kernel: no memset node, usable in captured work)
int launch_fill_u32(uint32_t *p, uint32_t v, uint64_t count, void *stream);
int launch_peak(const uint32_t *tab, uint32_t steps, uint32_t *out, int D, int blocks, void *stream);
// register-only XOR + popcount ceiling, variant v < kPeakVariants: blocks x
// 256 lanes, each doing steps x items x words 32-bit XOR+popcount
// operations (peak_reg_shape); steps a multiple of 4; out holds one word per
// lane
constexpr int kPeakVariants = 4;
int peak_reg_shape(int v, int *items, int *words);
int launch_peak_reg(int v, uint32_t steps, uint32_t seed, uint32_t *out, int blocks, void *stream);

// Split of the w rows of a pair between the levels, chosen identically by
// the host planner and the persistent batch scheduler.  The balanced
// two-level split (b = min(w/2, bcap)) is kept while a typical left subset
// (maximum e at the expected position (k-b)a/(a+1)) has at least
// kSplitShortRun right entries.  Otherwise the right side takes a second
// table level of b2 = bcap rows (min(bcap, w-2) unless fixed_b2) and the
// smallest left size a that still gives kSplitMinItems left subsets, no
// more than kSplitMaxInner inner entries per outer entry on average, and no
// more than kSplitMaxInnerWorst inner entries behind any single outer entry
// (the lowest Y1, right above the lowest left subset: C(k-a-b1, b2)).  A
// chunk holds whole inner ranges, so that worst range bounds the work one
// wave can be stuck with while the rest of the pair waits.
constexpr uint64_t kSplitShortRun = 256;
constexpr uint64_t kSplitMinItems = 2048;
constexpr uint64_t kSplitMaxInner = 4096;
constexpr uint64_t kSplitMaxInnerWorst = 1u << 15;
constexpr uint64_t kSplitMinRun = 64;

template <class BinomFn>
MD_HD inline void split_rows(int k, int w, int bcap, bool fixed_b2, const BinomFn &C,
                             int &a, int &b, int &b2, uint64_t min_items = 0) {
    b = w / 2 < bcap ? w / 2 : bcap;
    a = w - b;
    b2 = 0;
    // a launch for one pair alone: if the balanced split leaves fewer than
    // min_items left subsets (too few to keep every wave busy), move rows to
    // the left side while the typical right run keeps kSplitMinRun entries
    if (min_items && C(k - b, a) < min_items) {
        bool moved = false;
        while (b > 1 && C(k - b, a) < min_items) {
            const int e2 = (k - (b - 1)) * (a + 1) / (a + 2);
            if (C(k - 1 - e2, b - 1) < kSplitMinRun) break;
            --b;
            ++a;
            moved = true;
        }
        if (moved) return;
    }
    if (w < 5) return;
    const int e_typ = (k - b) * a / (a + 1);
    if (C(k - 1 - e_typ, b) >= kSplitShortRun) return;
    const int s2 = fixed_b2 ? bcap : (bcap < w - 2 ? bcap : w - 2);
    if (s2 < 1 || s2 > w - 2) return;
    for (int aa = 1; aa <= w - 2; ++aa) {
        const int b1 = w - aa - s2;
        if (b1 < 1) break;
        if (b1 > bcap) continue;
        if (C(k - b1 - s2, aa) < kSplitMinItems) continue;
        if (C(k - aa - b1, s2) > kSplitMaxInnerWorst) continue;
        const int e = (k - b1 - s2) * aa / (aa + 1);
        const uint64_t outer = C(k - 1 - s2 - e, b1);
        const uint64_t both = C(k - 1 - e, b1 + s2);
        if (outer == 0 || both / outer > kSplitMaxInner) continue;
        a = aa;
        b = b1;
        b2 = s2;
        return;
    }
}

}  // namespace md
