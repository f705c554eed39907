/*
 * mindist_oracle.c -- plain CPU oracle for the minimum distance of a binary
 * linear code (Hernando, Igual, Quintana-Orti, "Fast Algorithms for the
 * Computation of the Minimum Distance of a Random Linear Code").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code with the HIP path.
 *
 * What it computes, each function citing the passage it follows:
 *   orc_brute      -- the plain definition (Section 2: d(C) = wt(C) = minimum
 *                     weight of a nonzero codeword), by walking all 2^k
 *                     messages in binary-reflected Gray order; also the
 *                     full weight distribution.
 *   orc_partition  -- disjoint information sets (Section 2, the paragraph
 *                     introducing Gamma_1..Gamma_m): greedy rounds over the
 *                     still-unused columns in ascending order.
 *   orc_gamma      -- the systematic matrix of one information set: the
 *                     reduced row echelon form of G under the column order
 *                     (set columns ascending, then all others ascending).
 *   orc_pair       -- min / sum / count of wt(c Gamma) over all c with
 *                     wt(c) = g (Algorithm 1, the inner minimum), enumerating
 *                     combinations in lexicographic order with a stack of
 *                     prefix sums (Section 3.3, stack-based algorithm).
 *   orc_bz         -- Algorithm 1 (Brouwer-Zimmerman level loop) with the
 *                     lower bound of Section 2.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - partition: greedy ascending rounds; the columns left after the last
 *     full round form the partial set, whose rank k_m may be 0;
 *   - partial-set basis: full reduction makes it unique;
 *   - termination: by default L is raised after every Gamma_j ("one after
 *     each Gamma_j"), L_{j,g} = sum_{i<=j} f_i(g) + sum_{i>j} f_i(g-1) with
 *     f_full(h) = h+1 and f_partial(h) = max(0, h+1-(k-k_m)); the literal
 *     per-level update of Algorithm 1 is available as an option;
 *   - the partial set is enumerated at every level (literal loop j=1..m)
 *     unless an option drops it together with its bound term, or defers it
 *     to the first level g whose term max(0, g+1-(k-k_m)) is positive; the
 *     term bounds the set's columns only for codewords whose message under
 *     Gamma_m weighs more than every level enumerated, so that first level
 *     also enumerates the set's lower levels (ascending, after the full sets);
 *   - L starts at 1, U at n-k+1 (Algorithm 1, first line); a witness only
 *     comes from an enumerated codeword; U_found only moves on a strictly
 *     smaller weight; the witness is the first codeword reaching the final
 *     weight in (pair order, lexicographic rank) order.
 *
 * Words: rows are k x W uint64, column c at bit c%64 of word c/64.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define ORC_MAXW 8
#define ORC_MAXG 64

enum { ORC_OK = 0, ORC_E_ARG = -1, ORC_E_RANK = -2, ORC_E_NOMEM = -4,
       ORC_E_LIMIT = -6 };

/*
 * Planted mistakes, for the tests that show the pins catch them (0 = none,
 * the only value outside those tests):
 *   1 full sets contribute h instead of h+1 to the lower bound (a dropped term)
 *   2 every set is counted at level g in the per-pair bound (a wrong index)
 *   3 each pair stops one combination early
 *   4 Gamma_j is reduced only below each pivot (not the reduced echelon form)
 *   5 the weight ignores the last word of a codeword
 *   6 pivots found after the set's own columns (the lower block of the
 *     partial set) clear their column only in the rows below them
 *   7 a partial set deferred to its first useful level enumerates only that
 *     level, yet its bound term counts as if its lower levels were done
 */
static int orc_fault = 0;
void orc_set_fault(int f) { orc_fault = f; }

static int popw(const uint64_t *x, int W)
{
    int s = 0;
    for (int i = 0; i < W - (orc_fault == 5 && W > 1 ? 1 : 0); i++) s += __builtin_popcountll(x[i]);
    return s;
}

static int getbit(const uint64_t *row, int c) { return (int)((row[c >> 6] >> (c & 63)) & 1u); }

/* binomial coefficient, saturating at UINT64_MAX */
uint64_t orc_binom(int n, int r)
{
    if (r < 0 || n < 0 || r > n) return 0;
    if (r > n - r) r = n - r;
    unsigned __int128 v = 1;
    for (int i = 1; i <= r; i++) {
        v = v * (unsigned)(n - r + i) / (unsigned)i;   /* exact at every step */
        if (v > (unsigned __int128)UINT64_MAX) return UINT64_MAX;
    }
    return (uint64_t)v;
}

static int check_args(const uint64_t *G, int n, int k)
{
    if (!G || k < 1 || n <= k || n > 512) return ORC_E_ARG;
    int W = (n + 63) / 64;
    int rem = n - 64 * (W - 1);
    if (rem < 64)
        for (int r = 0; r < k; r++)
            if (G[(size_t)r * W + W - 1] >> rem) return ORC_E_ARG;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Plain definition: all 2^k - 1 nonzero messages, one row addition per  */
/* step along the binary-reflected Gray code.                            */
/* dist[w] = number of messages whose codeword has weight w (n+1 slots). */
/* Returns d, or a negative error (rank < k gives ORC_E_RANK).           */
/* ------------------------------------------------------------------ */
int orc_brute(const uint64_t *G, int n, int k, uint64_t *dist, uint64_t *witness)
{
    int e = check_args(G, n, k);
    if (e) return e;
    if (k > 30) return ORC_E_LIMIT;
    int W = (n + 63) / 64;
    uint64_t x[ORC_MAXW] = {0};
    if (dist) memset(dist, 0, sizeof(uint64_t) * (size_t)(n + 1));
    if (dist) dist[0] = 1;
    int best = n + 1;
    uint64_t total = (uint64_t)1 << k;
    for (uint64_t i = 1; i < total; i++) {
        int b = __builtin_ctzll(i);             /* Gray code flips message bit b */
        const uint64_t *row = G + (size_t)b * W;
        for (int t = 0; t < W; t++) x[t] ^= row[t];
        int w = popw(x, W);
        if (w == 0) return ORC_E_RANK;         /* a nonzero message maps to 0 */
        if (dist) dist[w]++;
        if (w < best) {
            best = w;
            if (witness) memcpy(witness, x, sizeof(uint64_t) * W);
        }
    }
    return best;
}

/* ------------------------------------------------------------------ */
/* Information sets.                                                      */
/* A column is viewed as a k-bit vector; independence is tested against an */
/* XOR basis indexed by leading bit (Gaussian elimination on columns).      */
/* sets_out receives the columns of S_1..S_mfull (k each, ascending) then   */
/* the k_m columns of the partial set (ascending).                          */
/* ------------------------------------------------------------------ */
typedef struct { uint64_t v[ORC_MAXW]; } colvec;

static void column_of(const uint64_t *G, int W, int k, int c, colvec *out)
{
    memset(out, 0, sizeof(*out));
    for (int r = 0; r < k; r++)
        if (getbit(G + (size_t)r * W, c)) out->v[r >> 6] |= (uint64_t)1 << (r & 63);
}

static int lead_bit(const colvec *x, int KW)
{
    for (int t = KW - 1; t >= 0; t--)
        if (x->v[t]) return 64 * t + 63 - __builtin_clzll(x->v[t]);
    return -1;
}

/* try to add x to the basis; returns 1 if x was independent */
static int basis_insert(colvec *basis, int *have, colvec x, int KW)
{
    for (;;) {
        int lb = lead_bit(&x, KW);
        if (lb < 0) return 0;
        if (!have[lb]) { basis[lb] = x; have[lb] = 1; return 1; }
        for (int t = 0; t < KW; t++) x.v[t] ^= basis[lb].v[t];
    }
}

int orc_partition(const uint64_t *G, int n, int k, int *sets_out, int *m_full, int *k_m)
{
    int e = check_args(G, n, k);
    if (e) return e;
    int W = (n + 63) / 64, KW = (k + 63) / 64;
    int *avail = malloc(sizeof(int) * n), navail = n;
    colvec *basis = malloc(sizeof(colvec) * k);
    int *have = malloc(sizeof(int) * k);
    int *piv = malloc(sizeof(int) * k);
    if (!avail || !basis || !have || !piv) { free(avail); free(basis); free(have); free(piv); return ORC_E_NOMEM; }
    for (int c = 0; c < n; c++) avail[c] = c;
    int mf = 0, out = 0, km = 0, first = 1;
    for (;;) {
        memset(have, 0, sizeof(int) * k);
        int np = 0;
        for (int i = 0; i < navail && np < k; i++) {
            colvec x;
            column_of(G, W, k, avail[i], &x);
            if (basis_insert(basis, have, x, KW)) piv[np++] = avail[i];
        }
        if (first && np < k) { free(avail); free(basis); free(have); free(piv); return ORC_E_RANK; }
        first = 0;
        if (np == k) {
            for (int i = 0; i < k; i++) sets_out[out++] = piv[i];
            mf++;
            /* remove the pivots from avail (both lists ascending) */
            int w = 0, p = 0;
            for (int i = 0; i < navail; i++) {
                if (p < k && avail[i] == piv[p]) { p++; continue; }
                avail[w++] = avail[i];
            }
            navail = w;
            if (navail == 0) break;
        } else {
            for (int i = 0; i < np; i++) sets_out[out++] = piv[i];
            km = np;
            break;
        }
    }
    *m_full = mf;
    *k_m = km;
    free(avail); free(basis); free(have); free(piv);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Reduced row echelon form of G under the column order                   */
/* (first[0..nfirst) ascending, then every other column ascending).         */
/* Output rows keep the original column positions.  The first nfirst        */
/* columns must be independent (they are when they come from partition).    */
/* ------------------------------------------------------------------ */
int orc_gamma(const uint64_t *G, int n, int k, const int *first, int nfirst, uint64_t *Gamma)
{
    int e = check_args(G, n, k);
    if (e) return e;
    int W = (n + 63) / 64;
    int *order = malloc(sizeof(int) * n);
    char *infirst = calloc(n, 1);
    if (!order || !infirst) { free(order); free(infirst); return ORC_E_NOMEM; }
    int no = 0;
    for (int i = 0; i < nfirst; i++) { order[no++] = first[i]; infirst[first[i]] = 1; }
    for (int c = 0; c < n; c++) if (!infirst[c]) order[no++] = c;
    memcpy(Gamma, G, sizeof(uint64_t) * (size_t)k * W);
    int r = 0;
    for (int oi = 0; oi < n && r < k; oi++) {
        int c = order[oi];
        int p = -1;
        for (int i = r; i < k; i++) if (getbit(Gamma + (size_t)i * W, c)) { p = i; break; }
        if (p < 0) {
            if (oi < nfirst) { free(order); free(infirst); return ORC_E_RANK; }
            continue;
        }
        if (p != r)
            for (int t = 0; t < W; t++) {
                uint64_t tmp = Gamma[(size_t)p * W + t];
                Gamma[(size_t)p * W + t] = Gamma[(size_t)r * W + t];
                Gamma[(size_t)r * W + t] = tmp;
            }
        int from = (orc_fault == 4 || (orc_fault == 6 && oi >= nfirst)) ? r + 1 : 0;
        for (int i = from; i < k; i++)
            if (i != r && getbit(Gamma + (size_t)i * W, c))
                for (int t = 0; t < W; t++) Gamma[(size_t)i * W + t] ^= Gamma[(size_t)r * W + t];
        r++;
    }
    free(order); free(infirst);
    return r == k ? ORC_OK : ORC_E_RANK;
}

/* ------------------------------------------------------------------ */
/* One pair: every g-subset of the k rows, lexicographic order.           */
/* ------------------------------------------------------------------ */

/* lexicographic rank -> combination: position i takes the smallest value v */
/* such that fewer than rank combinations start with a smaller value there. */
static void lex_unrank(uint64_t rank, int k, int g, int *c)
{
    int v = 0;
    for (int i = 0; i < g; i++) {
        for (;;) {
            uint64_t cnt = orc_binom(k - 1 - v, g - 1 - i);   /* combos with c_i = v */
            if (rank < cnt) break;
            rank -= cnt;
            v++;
        }
        c[i] = v++;
    }
}

typedef struct {
    int minw;              /* n+1 if nothing enumerated */
    uint64_t min_rank;     /* lexicographic rank of the first minimum */
    uint64_t wsum, count, adds;
} pair_acc;

typedef struct {
    const uint64_t *Gamma;
    int n, k, g, W;
    uint64_t lo, hi, chunk;
    uint64_t next;                 /* shared cursor (protected by mu) */
    pthread_mutex_t mu;
    pair_acc acc;
} pair_job;

static void acc_merge(pair_acc *into, const pair_acc *a)
{
    if (a->minw < into->minw || (a->minw == into->minw && a->min_rank < into->min_rank)) {
        into->minw = a->minw;
        into->min_rank = a->min_rank;
    }
    into->wsum += a->wsum;
    into->count += a->count;
    into->adds += a->adds;
}

/* Walk `len` combinations starting at lexicographic rank `start`.          */
/* stack[t] holds the sum of rows c_0..c_t (stack-based algorithm); after a */
/* successor step that changes position i, levels i..g-1 are rebuilt.       */
static void walk_range(const pair_job *jb, uint64_t start, uint64_t len, pair_acc *acc)
{
    int k = jb->k, g = jb->g, W = jb->W;
    int c[ORC_MAXG];
    uint64_t stack[ORC_MAXG][ORC_MAXW];
    lex_unrank(start, k, g, c);
    for (int t = 0; t < g; t++)
        for (int x = 0; x < W; x++)
            stack[t][x] = (t ? stack[t - 1][x] : 0) ^ jb->Gamma[(size_t)c[t] * W + x];
    acc->adds += (uint64_t)(g - 1);
    uint64_t rank = start;
    for (uint64_t s = 0; s < len; s++, rank++) {
        int w = popw(stack[g - 1], W);
        acc->wsum += (uint64_t)w;
        acc->count++;
        if (w < acc->minw) { acc->minw = w; acc->min_rank = rank; }
        if (s + 1 == len) break;
        if (orc_fault == 3 && s + 2 == len && start + len >= orc_binom(k, g)) break;
        int i = g - 1;
        while (i >= 0 && c[i] == k - g + i) i--;
        if (i < 0) break;
        c[i]++;
        for (int t = i + 1; t < g; t++) c[t] = c[t - 1] + 1;
        for (int t = i; t < g; t++)
            for (int x = 0; x < W; x++)
                stack[t][x] = (t ? stack[t - 1][x] : 0) ^ jb->Gamma[(size_t)c[t] * W + x];
        acc->adds += (uint64_t)(i ? g - i : g - 1);
    }
}

static void *pair_worker(void *arg)
{
    pair_job *jb = arg;
    pair_acc local = { jb->n + 1, 0, 0, 0, 0 };
    for (;;) {
        pthread_mutex_lock(&jb->mu);
        uint64_t s = jb->next;
        if (s < jb->hi) jb->next = (jb->hi - s > jb->chunk) ? s + jb->chunk : jb->hi;
        uint64_t e = jb->next;
        pthread_mutex_unlock(&jb->mu);
        if (s >= jb->hi) break;
        walk_range(jb, s, e - s, &local);
    }
    pthread_mutex_lock(&jb->mu);
    acc_merge(&jb->acc, &local);
    pthread_mutex_unlock(&jb->mu);
    return NULL;
}

/* min / argmin-rank / weight sum / count / row additions of wt(c Gamma) over */
/* the g-subsets c with lexicographic rank in [lo, hi).  hi is clamped to     */
/* C(k,g).  Returns the minimum weight (n+1 if the range is empty).           */
int orc_pair(const uint64_t *Gamma, int n, int k, int g, uint64_t lo, uint64_t hi,
             int threads, uint64_t *min_rank, uint64_t *wsum, uint64_t *count, uint64_t *adds)
{
    if (!Gamma || k < 1 || n < 1 || n > 512 || g < 1 || g > k || g > ORC_MAXG) return ORC_E_ARG;
    uint64_t total = orc_binom(k, g);
    if (total == UINT64_MAX) return ORC_E_LIMIT;
    if (hi > total) hi = total;
    pair_job jb;
    memset(&jb, 0, sizeof(jb));
    jb.Gamma = Gamma; jb.n = n; jb.k = k; jb.g = g; jb.W = (n + 63) / 64;
    jb.lo = lo; jb.hi = hi; jb.next = lo; jb.chunk = (uint64_t)1 << 20;
    jb.acc.minw = n + 1;
    pthread_mutex_init(&jb.mu, NULL);
    if (threads < 1) threads = 1;
    if (lo < hi) {
        if (threads == 1 || hi - lo <= jb.chunk) {
            walk_range(&jb, lo, hi - lo, &jb.acc);
        } else {
            pthread_t *th = malloc(sizeof(pthread_t) * threads);
            if (!th) { pthread_mutex_destroy(&jb.mu); return ORC_E_NOMEM; }
            for (int t = 0; t < threads; t++) pthread_create(&th[t], NULL, pair_worker, &jb);
            for (int t = 0; t < threads; t++) pthread_join(th[t], NULL);
            free(th);
        }
    }
    pthread_mutex_destroy(&jb.mu);
    if (min_rank) *min_rank = jb.acc.min_rank;
    if (wsum) *wsum = jb.acc.wsum;
    if (count) *count = jb.acc.count;
    if (adds) *adds = jb.acc.adds;
    return jb.acc.minw;
}

/* codeword of the g-subset with lexicographic rank `rank` */
int orc_combo_codeword(const uint64_t *Gamma, int n, int k, int g, uint64_t rank, int *combo, uint64_t *word)
{
    int W = (n + 63) / 64;
    int c[ORC_MAXG];
    if (g < 1 || g > k || g > ORC_MAXG || rank >= orc_binom(k, g)) return ORC_E_ARG;
    lex_unrank(rank, k, g, c);
    memset(word, 0, sizeof(uint64_t) * W);
    for (int i = 0; i < g; i++) {
        if (combo) combo[i] = c[i];
        for (int x = 0; x < W; x++) word[x] ^= Gamma[(size_t)c[i] * W + x];
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1.                                                           */
/* ------------------------------------------------------------------ */
typedef struct {
    int term_per_level;      /* 0: raise L after every Gamma_j; 1: literal per-level update */
    int partial_policy;      /* 0: partial set at every level; 1: dropped with its bound
                                term; 2: from the first level its term is positive */
    int threads;
} orc_opts;

/* bound contribution of set j after its level h has been enumerated */
static int f_bound(int j, int h, int m_full, int k, int k_m)
{
    if (j < m_full) return orc_fault == 1 ? h : h + 1;
    int v = h + 1 - (k - k_m);
    return v > 0 ? v : 0;
}

/*
 * Outputs (caller-owned):
 *   sets       n ints: columns of S_1..S_mfull, then the partial set
 *   counts     nsets_cap*(k+1) uint64: combinations enumerated for pair (j,g)
 *   pair_min   nsets_cap*(k+1) int: minimum weight of pair (j,g), -1 if not visited
 *   wsum       nsets_cap*(k+1) uint64: sum of the weights of pair (j,g)
 *   trace      up to trace_cap entries of 6 ints per visited pair:
 *              (j, h, L_before, L_after, U_after, pair_min), h the level the
 *              pair enumerates (h = g except the partial set's lower levels
 *              enumerated late under policy 2); L_after includes the
 *              per-level update when the pair ends its level
 *   info       8 ints: d, m_full, k_m, n_gamma, pairs_visited, L_final, U_final, last level
 *   witness    W uint64; witness_combo: up to ORC_MAXG ints, witness_meta: (j, g, lex rank)
 */
int orc_bz(const uint64_t *G, int n, int k, const orc_opts *opt, int nsets_cap,
           int *sets, uint64_t *counts, int *pair_min, uint64_t *wsum,
           int *trace, int trace_cap, int *info, uint64_t *witness,
           int *witness_combo, uint64_t *witness_meta)
{
    int e = check_args(G, n, k);
    if (e) return e;
    int W = (n + 63) / 64;
    int m_full = 0, k_m = 0;
    e = orc_partition(G, n, k, sets, &m_full, &k_m);
    if (e) return e;
    int policy = opt ? opt->partial_policy : 0;
    int has_partial = (k_m >= 1) && policy != 1;
    int ng = m_full + (has_partial ? 1 : 0);
    if (ng > nsets_cap) return ORC_E_LIMIT;
    int threads = opt ? opt->threads : 1;
    int per_level = opt ? opt->term_per_level : 0;

    uint64_t *Gam = malloc(sizeof(uint64_t) * (size_t)ng * k * W);
    if (!Gam) return ORC_E_NOMEM;
    for (int j = 0; j < ng; j++) {
        int nf = (j < m_full) ? k : k_m;
        e = orc_gamma(G, n, k, sets + (size_t)j * k, nf, Gam + (size_t)j * k * W);
        if (e) { free(Gam); return e; }
    }
    size_t cells = (size_t)nsets_cap * (k + 1);
    memset(counts, 0, sizeof(uint64_t) * cells);
    memset(wsum, 0, sizeof(uint64_t) * cells);
    for (size_t i = 0; i < cells; i++) pair_min[i] = -1;

    int L = 1;
    int U_found = n + 1;            /* "infinity": no codeword found yet */
    int singleton = n - k + 1;
    int pairs = 0, last_g = 0;
    int wj = -1, wg = 0;
    uint64_t wrank = 0;
    /* last level enumerated per set; the pairs (set, level) of one level */
    int *done = calloc((size_t)ng, sizeof(int));
    int *pj = malloc(sizeof(int) * (size_t)(m_full + k + 1));
    int *ph = malloc(sizeof(int) * (size_t)(m_full + k + 1));
    if (!done || !pj || !ph) { free(done); free(pj); free(ph); free(Gam); return ORC_E_NOMEM; }
    for (int g = 1; g <= k; g++) {
        int U = U_found < singleton ? U_found : singleton;
        if (L >= U) break;
        if (g > ORC_MAXG) { free(done); free(pj); free(ph); free(Gam); return ORC_E_LIMIT; }
        /* the pairs of level g: every full set at level g, then the partial
           set at g, or under policy 2 (once its term at g is positive) at
           every level it has not done yet */
        int np = 0;
        for (int j = 0; j < m_full; j++) { pj[np] = j; ph[np] = g; np++; }
        if (has_partial) {
            if (policy == 0) { pj[np] = m_full; ph[np] = g; np++; }
            else if (g + 1 - (k - k_m) > 0)
                for (int h = (orc_fault == 7 ? g : done[m_full] + 1); h <= g; h++) {
                    pj[np] = m_full; ph[np] = h; np++;
                }
        }
        int stop = 0;
        for (int q = 0; q < np; q++) {
            int j = pj[q], h = ph[q];
            U = U_found < singleton ? U_found : singleton;
            if (!per_level && L >= U) { stop = 1; break; }
            int Lb = L;
            uint64_t mr = 0, ws = 0, cnt = 0;
            int pm = orc_pair(Gam + (size_t)j * k * W, n, k, h, 0, UINT64_MAX, threads, &mr, &ws, &cnt, NULL);
            if (pm < 0) { free(done); free(pj); free(ph); free(Gam); return pm; }
            counts[(size_t)j * (k + 1) + h] = cnt;
            wsum[(size_t)j * (k + 1) + h] = ws;
            pair_min[(size_t)j * (k + 1) + h] = pm;
            done[j] = h;
            if (pm < U_found) { U_found = pm; wj = j; wg = h; wrank = mr; }
            /* the bound from the levels each set has done: after every pair,
               or only at the end of the level (literal per-level rule) */
            if (!per_level || q == np - 1) {
                int s = 0;
                for (int i = 0; i < ng; i++)
                    s += f_bound(i, (orc_fault == 2 && i < m_full) ? g : done[i], m_full, k, k_m);
                L = s;
            }
            U = U_found < singleton ? U_found : singleton;
            if (trace && pairs < trace_cap) {
                int *t = trace + 6 * pairs;
                t[0] = j; t[1] = h; t[2] = Lb; t[3] = L; t[4] = U; t[5] = pm;
            }
            pairs++;
            last_g = g;
        }
        if (stop) break;
    }
    free(done); free(pj); free(ph);
    int U = U_found < singleton ? U_found : singleton;
    if (info) {
        info[0] = U; info[1] = m_full; info[2] = k_m; info[3] = ng;
        info[4] = pairs; info[5] = L; info[6] = U_found; info[7] = last_g;
    }
    if (wj >= 0) {
        int combo[ORC_MAXG];
        orc_combo_codeword(Gam + (size_t)wj * k * W, n, k, wg, wrank, combo, witness);
        if (witness_combo) memcpy(witness_combo, combo, sizeof(int) * wg);
        if (witness_meta) { witness_meta[0] = (uint64_t)wj; witness_meta[1] = (uint64_t)wg; witness_meta[2] = wrank; }
    }
    free(Gam);
    return ORC_OK;
}
