// mindist_plan.h -- host-side mathematics shared by the single-code,
// batch and serving paths: binomials, argument checks, information sets and
// systematic matrices (Section 2), the lower-bound schedule (Section 2 and
// Algorithm 1), colex unranking and row packing.
//
// Readings of the paper implemented here:
//   * information sets: greedy rounds over the unused columns in ascending
//     order; a round that reaches k pivots is a full set, the first round
//     that does not gives the partial set (rank k_m, possibly 0) and ends;
//   * Gamma_j: the reduced row echelon form of G under the column order
//     (set columns ascending, then all others ascending) -- unique, so the
//     partial set's [[I, A], [0, B]] is canonical;
//   * bounds: U starts at n-k+1, L at 1 (Algorithm 1); after pair (j, w),
//     L = sum_{i<=j} f_i(w) + sum_{i>j} f_i(w-1) with f_full(h) = h+1 and
//     f_partial(h) = max(0, h+1-(k-k_m)) ("one after each Gamma_j").
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace md {

// records msg as the calling thread's last error and returns code
int fail(int code, const std::string &msg);

struct Binom {
    std::vector<uint64_t> t;   // kBinomX x kBinomT, saturating at UINT64_MAX
    Binom();
    uint64_t operator()(int x, int r) const;
};
const Binom &BN();

// default cap on one saved-sum table of the single-code path: 1 GiB keeps
// six-row right tables of k ~ 51 (576 MB at 8 words per entry), whose longer
// right runs lift the w >= 12 pairs of such codes by 4-12 %
constexpr uint64_t kTableCapDefault = 1ull << 30;

inline uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
inline int bit_of(const uint64_t *row, int c) { return (int)((row[c >> 6] >> (c & 63)) & 1u); }
inline int dp_of_host(int D) { return D <= 1 ? 1 : D <= 2 ? 2 : D <= 4 ? 4 : D <= 8 ? 8 : 16; }

int check_matrix(const uint64_t *G, int n, int k);

struct Plan {
    int n = 0, k = 0, W = 0;
    int m_full = 0, k_m = 0;
    std::vector<std::vector<int>> sets;          // full sets, then the partial set
    std::vector<std::vector<uint64_t>> gamma;    // k x W rows per set, original columns
};
int make_plan(const uint64_t *G, int n, int k, Plan &P);

// the columns a set's rows carry on the device: the non-set columns for a
// full set (its identity part is implied by the level), all columns for the
// partial set
std::vector<int> carried_columns(const Plan &P, int j);
// pack the carried columns of one Gamma row into 32-bit words
void pack_row(const uint64_t *row, const std::vector<int> &cols, uint32_t *out, int DP);

int bound_f(int i, int h, int m_full, int k, int k_m);
int bound_after(int k, int m_full, int k_m, int n_gamma, int j, int w);

// colex unranking of rho into an r-subset of [0, hi) (elements ascending)
void colex_unrank(uint64_t rho, int r, int hi, int *out);

// How one pair's w-subsets are split (see mindist_internal.h): a rows per
// lane, b rows from the (outer) right table, b2 rows from the inner table
// (0: two-level).  The two-level split b = min(w/2, bcap) is kept unless a
// lane subset would typically meet fewer than 1024 right entries; then the
// three-level split with b2 = min(bcap, w-2) (fixed_b2: exactly bcap) and the
// smallest a leaving at least 2048 lane subsets.
struct Split { int a, b, b2; };
// min_items > 0: a pair launched alone; favour at least that many left
// subsets (see split_rows)
Split choose_split(int k, int w, int bcap, bool fixed_b2, uint64_t min_items = 0);
// outer-table entries per chunk of a three-level pair: about 256K codewords
// per chunk of tile_items lane subsets
uint32_t outer_tile(int k, const Split &sp, uint32_t tile_items);
// rows of the witness recorded in a slot (ascending); empty if invalid
struct Slot;
std::vector<int> witness_rows(int k, int a, int b, int b2, const Slot &s);

}  // namespace md
