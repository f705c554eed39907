// mindist_plan.cpp -- host-side mathematics shared by all paths (see
// mindist_plan.h for the readings of the paper it implements).
#include "mindist_plan.h"

#include <algorithm>
#include <cstring>
#include <iterator>
#include <string>

#include "../../include/mindist.h"
#include "mindist_internal.h"

namespace md {

static thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

const char *last_error_text() { return g_err.c_str(); }


Binom::Binom() : t((size_t)kBinomX * kBinomT, 0) {
        for (int x = 0; x < kBinomX; ++x) {
            t[(size_t)x * kBinomT] = 1;
            for (int r = 1; r < kBinomT; ++r) {
                if (r > x) { t[(size_t)x * kBinomT + r] = 0; continue; }
                uint64_t a = t[(size_t)(x - 1) * kBinomT + r - 1];
                uint64_t b = (r <= x - 1) ? t[(size_t)(x - 1) * kBinomT + r] : 0;
                uint64_t s = a + b;
                t[(size_t)x * kBinomT + r] = (s < a || a == UINT64_MAX || b == UINT64_MAX) ? UINT64_MAX : s;
            }
        }
}

uint64_t Binom::operator()(int x, int r) const {
    if (x < 0 || r < 0 || r > x) return 0;
    if (x >= kBinomX || r >= kBinomT) return UINT64_MAX;
    return t[(size_t)x * kBinomT + r];
}
const Binom &BN() {
    static Binom b;
    return b;
}

int check_matrix(const uint64_t *G, int n, int k) {
    if (!G) return fail(MINDIST_E_ARG, "G is NULL");
    if (k < 1 || n <= k || n > MINDIST_MAX_N)
        return fail(MINDIST_E_ARG, "need 1 <= k < n <= 512 (got n=" + std::to_string(n) +
                                       ", k=" + std::to_string(k) + ")");
    const int W = (n + 63) / 64;
    const int rem = n - 64 * (W - 1);
    if (rem < 64)
        for (int r = 0; r < k; ++r)
            if (G[(size_t)r * W + W - 1] >> rem)
                return fail(MINDIST_E_ARG, "bits beyond column n-1 must be zero (row " +
                                               std::to_string(r) + ")");
    return MINDIST_OK;
}

// One Gauss-Jordan sweep: pivot the columns of `cols` in order on rows r..k-1
// of M (k x W), eliminating every other row; stop at k pivots.  Appends the
// pivot columns and returns the new pivot row count.
static int sweep(std::vector<uint64_t> &M, int k, int W, const std::vector<int> &cols, int r,
          std::vector<int> *piv) {
    for (int c : cols) {
        if (r == k) break;
        int p = -1;
        for (int i = r; i < k; ++i)
            if (bit_of(&M[(size_t)i * W], c)) { p = i; break; }
        if (p < 0) continue;
        if (p != r)
            for (int t = 0; t < W; ++t) std::swap(M[(size_t)p * W + t], M[(size_t)r * W + t]);
        for (int i = 0; i < k; ++i)
            if (i != r && bit_of(&M[(size_t)i * W], c))
                for (int t = 0; t < W; ++t) M[(size_t)i * W + t] ^= M[(size_t)r * W + t];
        if (piv) piv->push_back(c);
        ++r;
    }
    return r;
}

int make_plan(const uint64_t *G, int n, int k, Plan &P) {
    int e = check_matrix(G, n, k);
    if (e) return e;
    const int W = (n + 63) / 64;
    P = Plan();
    P.n = n; P.k = k; P.W = W;
    std::vector<int> avail(n);
    for (int c = 0; c < n; ++c) avail[c] = c;
    bool first = true;
    for (;;) {
        std::vector<uint64_t> M(G, G + (size_t)k * W);
        std::vector<int> piv;
        int r = sweep(M, k, W, avail, 0, &piv);
        if (first && r < k) return fail(MINDIST_E_RANK, "rank(G) < k");
        first = false;
        if (r == k) {
            P.sets.push_back(piv);
            P.gamma.push_back(M);
            ++P.m_full;
            std::vector<int> rest;
            std::set_difference(avail.begin(), avail.end(), piv.begin(), piv.end(),
                                std::back_inserter(rest));
            avail.swap(rest);
            if (avail.empty()) break;
        } else {
            P.k_m = r;
            if (r >= 1) {
                // complete the echelon form on the remaining rows over all
                // other columns in ascending order
                std::vector<int> others;
                std::vector<int> s = piv;
                std::sort(s.begin(), s.end());
                for (int c = 0; c < n; ++c)
                    if (!std::binary_search(s.begin(), s.end(), c)) others.push_back(c);
                int r2 = sweep(M, k, W, others, r, nullptr);
                if (r2 != k) return fail(MINDIST_E_RANK, "rank(G) < k");
                P.sets.push_back(piv);
                P.gamma.push_back(M);
            }
            break;
        }
    }
    return MINDIST_OK;
}

int bound_f(int i, int h, int m_full, int k, int k_m) {
    if (i < m_full) return h + 1;
    int v = h + 1 - (k - k_m);
    return v > 0 ? v : 0;
}

int bound_after(int k, int m_full, int k_m, int n_gamma, int j, int w) {
    int s = 0;
    for (int i = 0; i < n_gamma; ++i) s += bound_f(i, i <= j ? w : w - 1, m_full, k, k_m);
    return s;
}

bool Schedule::next(const PairPos &p, PairPos *q) const {
    PairPos r = p;
    const int g0 = k - k_m;   // first level the partial term is positive
    if (p.j < m_full - 1) {
        r.j = p.j + 1;
        r.h = p.g;
    } else if (p.j == m_full - 1 && has_partial() &&
               (policy == kPartialAlways || p.g >= g0)) {
        r.j = m_full;
        r.h = (policy == kPartialWhenUseful && p.g == g0) ? 1 : p.g;
    } else if (p.j == m_full && p.h < p.g) {
        r.h = p.h + 1;
    } else {
        r.j = 0;
        r.g = p.g + 1;
        r.h = r.g;
    }
    if (r.g > k) return false;
    *q = r;
    return true;
}

bool Schedule::level_end(const PairPos &p) const {
    PairPos q;
    return !next(p, &q) || q.g != p.g;
}

int Schedule::bound_after(const PairPos &p) const {
    int s = 0;
    for (int i = 0; i < m_full; ++i) s += (i <= p.j) ? p.g + 1 : p.g;
    if (has_partial()) {
        // the level the partial set has done: h after its own pair, else the
        // previous level (its term is 0 below g0, so a set not started yet
        // under policy 2 counts the same)
        const int done = p.j == m_full ? p.h : p.g - 1;
        s += bound_f(m_full, done, m_full, k, k_m);
    }
    return s;
}

static int cert_fail(int t, const PairView &r, const std::string &what) {
    return fail(MINDIST_E_CERT, "certificate: pair " + std::to_string(t) + " (" + std::to_string(r.j) +
                                    "," + std::to_string(r.w) + "): " + what);
}

int certify_trace(const CertSpec &cs, const PairView *trace, int np, int d, int L_final,
                  int exited_midpair) {
    const Binom &B = BN();
    const Schedule &S = cs.sched;
    const int singleton = cs.n - cs.k + 1;
    const uint32_t kNone = 0xffffffffu;
    if (np < 1) return fail(MINDIST_E_CERT, "certificate: no pair visited");
    PairPos pos = S.first();
    bool more = true;
    int L = 1;
    uint32_t U_found = kNone;
    auto U_now = [&]() { return (int)std::min<uint32_t>(U_found, (uint32_t)singleton); };
    bool cut = false;
    for (int t = 0; t < np; ++t) {
        const PairView &r = trace[t];
        if (!more) return cert_fail(t, r, "beyond the last level");
        if (r.j != pos.j || r.w != pos.h)
            return cert_fail(t, r, "out of order, expected (" + std::to_string(pos.j) + "," +
                                       std::to_string(pos.h) + ")");
        if ((!cs.per_level || S.level_start(pos)) && L >= U_now())
            return cert_fail(t, r, "visited although L >= U before it");
        if (r.L_before != L)
            return cert_fail(t, r, "L before " + std::to_string(r.L_before) + ", expected " +
                                       std::to_string(L));
        if (r.count != B(cs.k, pos.h)) return cert_fail(t, r, "count is not C(k,w)");
        if (r.executed > r.count) return cert_fail(t, r, "more combinations evaluated than C(k,w)");
        if (r.executed > 0 && r.pair_min < 1) return cert_fail(t, r, "no least weight recorded");
        if (r.pair_min >= 0) U_found = std::min<uint32_t>(U_found, (uint32_t)r.pair_min);
        if (r.U_after != U_now())
            return cert_fail(t, r, "U after " + std::to_string(r.U_after) + ", expected " +
                                       std::to_string(U_now()));
        if (r.executed < r.count) {
            // mid-pair exit: the last pair only, and only once U <= L before it
            if (t != np - 1) return cert_fail(t, r, "cut short but not the last pair");
            if (!cs.midpair_exit || cs.per_level)
                return cert_fail(t, r, "cut short with mid-pair exit off");
            if (U_now() > L)
                return cert_fail(t, r, "cut short although U = " + std::to_string(U_now()) +
                                           " > L = " + std::to_string(L) + " before it");
            if (r.L_after != L) return cert_fail(t, r, "a cut pair raised L");
            cut = true;
            break;
        }
        const int La = S.L_after(pos, cs.per_level, L);
        if (r.L_after != La)
            return cert_fail(t, r, "L after " + std::to_string(r.L_after) + ", expected " +
                                       std::to_string(La));
        L = La;
        more = S.next(pos, &pos);
    }
    if (!cut && more && L < U_now())
        return fail(MINDIST_E_CERT, "certificate: stopped with L = " + std::to_string(L) + " < U = " +
                                        std::to_string(U_now()));
    if ((exited_midpair != 0) != cut) return fail(MINDIST_E_CERT, "certificate: mid-pair exit flag");
    if (d != U_now())
        return fail(MINDIST_E_CERT, "certificate: d = " + std::to_string(d) + " but U = " +
                                        std::to_string(U_now()));
    if (L_final != L)
        return fail(MINDIST_E_CERT, "certificate: final L = " + std::to_string(L_final) +
                                        ", expected " + std::to_string(L));
    if (U_found == kNone) return fail(MINDIST_E_CERT, "certificate: no codeword found");
    return MINDIST_OK;
}

int certify_witness(const Plan &P, int j, const std::vector<int> &rows, int w, int d,
                    uint64_t *word, uint64_t *row_mask) {
    const int W = P.W;
    if (j < 0 || j >= (int)P.gamma.size()) return fail(MINDIST_E_CERT, "witness names no set");
    if ((int)rows.size() != w) return fail(MINDIST_E_CERT, "witness decodes to an invalid combination");
    for (int t = 0; t < W; ++t) word[t] = 0;
    for (int t = 0; t < MINDIST_MAX_WORDS; ++t) row_mask[t] = 0;
    for (int r : rows) {
        if (r < 0 || r >= P.k) return fail(MINDIST_E_CERT, "witness names a row beyond k");
        for (int t = 0; t < W; ++t) word[t] ^= P.gamma[j][(size_t)r * W + t];
        row_mask[r >> 6] |= 1ull << (r & 63);
    }
    int wt = 0;
    for (int t = 0; t < W; ++t) wt += __builtin_popcountll(word[t]);
    if (wt != d)
        return fail(MINDIST_E_CERT, "witness weight " + std::to_string(wt) + " differs from d = " +
                                        std::to_string(d));
    // Gamma_0 is the identity on S_0: a codeword of the row space is the sum
    // of the rows its values on S_0 select
    std::vector<uint64_t> back(W, 0);
    for (int r = 0; r < P.k; ++r)
        if (bit_of(word, P.sets[0][r]))
            for (int t = 0; t < W; ++t) back[t] ^= P.gamma[0][(size_t)r * W + t];
    for (int t = 0; t < W; ++t)
        if (back[t] != word[t]) return fail(MINDIST_E_CERT, "witness is not in the row space of G");
    return MINDIST_OK;
}

// colex unranking of rho into an r-subset of [0, hi) (elements ascending)
void colex_unrank(uint64_t rho, int r, int hi, int *out) {
    const Binom &B = BN();
    for (int t = r; t >= 1; --t) {
        int lo = t - 1, h = hi - 1;
        while (lo < h) {
            int mid = (lo + h + 1) / 2;
            if (B(mid, t) <= rho) lo = mid; else h = mid - 1;
        }
        out[t - 1] = lo;
        rho -= B(lo, t);
        hi = lo;
    }
}


Split choose_split(int k, int w, int bcap, bool fixed_b2, uint64_t min_items) {
    const Binom &B = BN();
    Split sp{0, 0, 0};
    split_rows(k, w, bcap, fixed_b2, [&](int x, int r) { return B(x, r); }, sp.a, sp.b, sp.b2,
               min_items);
    return sp;
}

uint32_t outer_tile(int k, const Split &sp, uint32_t tile_items) {
    const Binom &B = BN();
    const int e = (k - sp.b - sp.b2) * sp.a / (sp.a + 1);
    const uint64_t outer = B(k - 1 - sp.b2 - e, sp.b);
    const uint64_t both = B(k - 1 - e, sp.b + sp.b2);
    const double n2 = outer ? (double)both / (double)outer : 1.0;
    const double want = 262144.0 / ((double)tile_items * (n2 > 1 ? n2 : 1));
    uint32_t T = 1;
    while (T < 1024 && T * 2 <= want) T <<= 1;
    return T;
}

std::vector<int> witness_rows(int k, int a, int b, int b2, const Slot &s) {
    int X[MINDIST_MAX_LEVEL + 1], Z[MINDIST_MAX_LEVEL + 1];
    colex_unrank(s.rho, a, k, X);
    colex_unrank(s.i, b, k - b2, Z);
    std::vector<int> rows(X, X + a);
    for (int t = 0; t < b; ++t) rows.push_back(k - 1 - b2 - Z[t]);
    if (b2) {
        colex_unrank(s.i2, b2, k, Z);
        for (int t = 0; t < b2; ++t) rows.push_back(k - 1 - Z[t]);
    }
    std::sort(rows.begin(), rows.end());
    if (std::adjacent_find(rows.begin(), rows.end()) != rows.end()) rows.clear();
    return rows;
}

std::vector<int> carried_columns(const Plan &P, int j) {
    std::vector<int> cols;
    if (j < P.m_full) {
        std::vector<int> s = P.sets[j];
        std::sort(s.begin(), s.end());
        for (int col = 0; col < P.n; ++col)
            if (!std::binary_search(s.begin(), s.end(), col)) cols.push_back(col);
    } else {
        for (int col = 0; col < P.n; ++col) cols.push_back(col);
    }
    return cols;
}

void pack_row(const uint64_t *row, const std::vector<int> &cols, uint32_t *out, int DP) {
    for (int d = 0; d < DP; ++d) out[d] = 0;
    for (size_t i = 0; i < cols.size(); ++i)
        if (bit_of(row, cols[i])) out[i >> 5] |= 1u << (i & 31);
}

}  // namespace md
