// mindist_walk.h -- the per-lane lexicographic walk over one pair (Gamma_j,
// w): a comparison kernel for the saved-sums enumeration (see
// mindist_walk.hip).  Host launcher and its argument block.
#pragma once
#include <stdint.h>

namespace md {

constexpr int kWalkMaxK = 128;   // rows staged in LDS
constexpr int kWalkMaxW = 12;    // subset size (partial sums kept in registers)
constexpr int kWalkMaxD = 4;     // carried 32-bit words per row

struct WalkOut {
    uint32_t min_weight;         // least weight found (0xFFFFFFFF before any)
    uint32_t pad;
    uint64_t executed;           // combinations evaluated
};

struct WalkArgs {
    const uint32_t *rows;        // k x dp_of(D) words, the carried columns of Gamma_j
    const uint64_t *binom;       // binomial table (kBinomX x kBinomT)
    WalkOut *out;
    uint64_t total;              // C(k, w)
    uint64_t per_thread;         // consecutive ranks per lane (the last lanes get fewer or none)
    int32_t k, w;
    uint32_t offset;             // weight of the stripped identity columns (w), else 0
};

// D in 1..kWalkMaxD; blocks of 256 threads; 0 on success
int launch_walk_pair(const WalkArgs &a, int D, int blocks, void *stream);

}  // namespace md
