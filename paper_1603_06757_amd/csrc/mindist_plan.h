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

// Algorithm 1's pair order and bounds (Section 2).  Level g visits every
// full set at level g, then the partial set (if k_m >= 1): at level g
// (policy 0, the literal loop over j = 1..m), never (policy 1, its bound
// term dropped too), or from the first level whose term
// max(0, g+1-(k-k_m)) is positive (policy 2): that term bounds the weight on
// the set's columns only once every level up to g is done under Gamma_m, so
// the first such level g0 = k-k_m also enumerates the set's levels 1..g0-1
// (ascending, after the full sets); later levels visit it at g only.
enum { kPartialAlways = 0, kPartialNever = 1, kPartialWhenUseful = 2 };
struct PairPos {
    int j = 0;   // set (full sets 0..m_full-1, partial set m_full)
    int h = 1;   // level the pair enumerates (= g except a catch-up pair)
    int g = 1;   // level of Algorithm 1's outer loop
};
struct Schedule {
    int k = 0, m_full = 0, k_m = 0, policy = kPartialAlways;
    Schedule() = default;
    Schedule(int k_, int m_full_, int k_m_, int policy_)
        : k(k_), m_full(m_full_), k_m(k_m_), policy(policy_) {}
    bool has_partial() const { return k_m >= 1 && policy != kPartialNever; }
    int n_sets() const { return m_full + (has_partial() ? 1 : 0); }
    PairPos first() const { return PairPos{}; }
    // the pair after p; false once the levels are exhausted (g > k)
    bool next(const PairPos &p, PairPos *q) const;
    // p is the last pair of its level
    bool level_end(const PairPos &p) const;
    // p opens its level (Algorithm 1's test under the per-level rule)
    bool level_start(const PairPos &p) const { return p.j == 0 && p.h == p.g; }
    // L once p completes: sum over sets of f_i(the level set i has done)
    int bound_after(const PairPos &p) const;
    // L after p under the termination rule (per_level: raised only when p
    // ends its level), given L before p
    int L_after(const PairPos &p, bool per_level, int L_before) const {
        return (!per_level || level_end(p)) ? bound_after(p) : L_before;
    }
};

// The certificate of a run (Section 2, Algorithm 1's termination): the
// visited pairs follow the schedule from L = 1, U = n-k+1; each pair covers
// C(k, h) combinations and every completed one evaluated exactly that many;
// L before, L after and U after each pair are the recomputed ones (U = the
// least pair minimum so far, capped at n-k+1); only the last pair may be
// cut short, and only when U <= L before it (mid-pair exit allowed); the
// run stopped because L >= U, because the last pair was cut, or because the
// levels ran out; d and L_final are the recomputed U and L.  Returns
// MINDIST_OK or MINDIST_E_CERT with the reason as last error.
struct CertSpec {
    int n = 0, k = 0;
    Schedule sched;
    bool per_level = false;
    bool midpair_exit = true;
};
struct PairView {   // the fields of a trace record the certificate reads
    int j, w, L_before, L_after, U_after, pair_min;
    uint64_t count, executed;
};
int certify_trace(const CertSpec &cs, const PairView *trace, int np, int d, int L_final,
                  int exited_midpair);
// The witness (Section 2): the XOR of the named rows of Gamma_j weighs d
// and lies in the row space of G (it equals the combination of Gamma_0's
// rows its own values on Gamma_0's information set select).  Writes the
// codeword (P.W words) and the row mask; MINDIST_E_CERT otherwise.
int certify_witness(const Plan &P, int j, const std::vector<int> &rows, int w, int d,
                    uint64_t *word, uint64_t *row_mask);

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
