/* mindist_cpu.c -- Section 3's CPU algorithms for one pair (Gamma, w): the
 * basic, optimized, stack-based and saved-additions enumerations (plus the
 * two-way unrolled saved variant), parallelised with OpenMP over the
 * outermost loop with a dynamic schedule.  Host baselines for measurement;
 * written from the section's descriptions, independent of the GPU library
 * and of the test oracle. */
#include "../../include/mindist_cpu.h"

#include <omp.h>
#include <stdlib.h>
#include <string.h>

#define MAXW 8        /* words per row */
#define MAXG 256      /* subset size bound (w <= k <= 256) */

typedef struct {
    int32_t min;
    uint64_t combos, adds;
} Acc;

static inline int weight_of(const uint64_t *x, int W) {
    int s = 0;
    for (int i = 0; i < W; ++i) s += __builtin_popcountll(x[i]);
    return s;
}

static inline void xor_into(uint64_t *dst, const uint64_t *a, const uint64_t *b, int W) {
    for (int i = 0; i < W; ++i) dst[i] = a[i] ^ b[i];
}

static uint64_t binom(int n, int r) {
    if (r < 0 || n < 0 || r > n) return 0;
    if (r > n - r) r = n - r;
    unsigned __int128 v = 1;
    for (int i = 1; i <= r; ++i) v = v * (unsigned)(n - r + i) / (unsigned)i;
    return v > (unsigned __int128)UINT64_MAX ? UINT64_MAX : (uint64_t)v;
}

static void merge(Acc *into, const Acc *a) {
    if (a->min < into->min) into->min = a->min;
    into->combos += a->combos;
    into->adds += a->adds;
}

/* the next combination after c (size m, elements of [0, k)) that keeps
 * c[0..fixed-1]; returns the changed position or -1 when none is left */
static int next_comb(int *c, int m, int k, int fixed) {
    int i = m - 1;
    while (i >= fixed && c[i] == k - m + i) --i;
    if (i < fixed) return -1;
    ++c[i];
    for (int j = i + 1; j < m; ++j) c[j] = c[j - 1] + 1;
    return i;
}

/* ---- Algorithm 2 ---------------------------------------------------- */
static void run_basic(const uint64_t *R, int k, int W, int w, int off, int nt, Acc *out) {
#pragma omp parallel num_threads(nt)
    {
        Acc a = {INT32_MAX, 0, 0};
#pragma omp for schedule(dynamic, 1)
        for (int f = 0; f <= k - w; ++f) {
            int c[MAXG];
            for (int i = 0; i < w; ++i) c[i] = f + i;
            do {
                uint64_t x[MAXW];
                memcpy(x, R + (size_t)c[0] * W, sizeof(uint64_t) * W);
                for (int i = 1; i < w; ++i) xor_into(x, x, R + (size_t)c[i] * W, W);
                a.adds += (uint64_t)(w - 1);
                const int wt = off + weight_of(x, W);
                if (wt < a.min) a.min = wt;
                ++a.combos;
            } while (next_comb(c, w, k, 1) >= 0);
        }
#pragma omp critical
        merge(out, &a);
    }
}

/* ---- Algorithms 3 and 4 --------------------------------------------- */
/* all combinations whose first w-1 elements sum to base: one addition each */
static inline void last_element(const uint64_t *R, int k, int W, int off, const uint64_t *base,
                                int from, Acc *a) {
    for (int e = from; e < k; ++e) {
        uint64_t x[MAXW];
        xor_into(x, base, R + (size_t)e * W, W);
        const int wt = off + weight_of(x, W);
        if (wt < a->min) a->min = wt;
    }
    a->combos += (uint64_t)(k - from);
    a->adds += (uint64_t)(k - from);
}

static void run_optimized(const uint64_t *R, int k, int W, int w, int off, int stack, int nt,
                          Acc *out) {
    const int m = w - 1;      /* size of the prefix combinations */
#pragma omp parallel num_threads(nt)
    {
        Acc a = {INT32_MAX, 0, 0};
#pragma omp for schedule(dynamic, 1)
        for (int f = 0; f <= k - w; ++f) {
            int c[MAXG];
            uint64_t S[MAXG][MAXW];   /* S[i] = rows c[0] + ... + c[i] */
            for (int i = 0; i < m; ++i) c[i] = f + i;
            memcpy(S[0], R + (size_t)f * W, sizeof(uint64_t) * W);
            for (int i = 1; i < m; ++i) xor_into(S[i], S[i - 1], R + (size_t)c[i] * W, W);
            a.adds += (uint64_t)(m - 1);
            for (;;) {
                last_element(R, k, W, off, S[m - 1], c[m - 1] + 1, &a);
                /* prefixes stay within rows 0..k-2: row k-1 could not be
                 * followed by a last element */
                const int p = next_comb(c, m, k - 1, 1);
                if (p < 0) break;
                if (stack) {
                    /* rebuild the stack from the leftmost changed element */
                    for (int i = p; i < m; ++i) xor_into(S[i], S[i - 1], R + (size_t)c[i] * W, W);
                    a.adds += (uint64_t)(m - p);
                } else {
                    /* the prefix sum from scratch */
                    memcpy(S[m - 1], R + (size_t)c[0] * W, sizeof(uint64_t) * W);
                    for (int i = 1; i < m; ++i) xor_into(S[m - 1], S[m - 1], R + (size_t)c[i] * W, W);
                    a.adds += (uint64_t)(m - 1);
                }
            }
        }
#pragma omp critical
        merge(out, &a);
    }
}

/* ---- Algorithm 5 ---------------------------------------------------- */
typedef struct {
    uint64_t n;          /* C(k, l) entries */
    uint64_t *sum;       /* n x W */
    uint8_t *last;       /* largest element of each subset */
} Level;

#define MAX_TABLE_BYTES (8ull << 30)   /* all saved levels of one pair */

/* level l in lexicographic order: for each first element x, row x plus the
 * level-(l-1) entries whose first element exceeds x (a suffix of that
 * level, since it is in lexicographic order too) */
static int build_levels(const uint64_t *R, int k, int W, int s, Level *L) {
    uint64_t bytes = 0;
    for (int l = 1; l <= s; ++l) {
        const uint64_t n = binom(k, l);
        if (n > (MAX_TABLE_BYTES / (8ull * W + 1))) return MINDIST_CPU_E_NOMEM;
        bytes += n * (8ull * W + 1);
    }
    if (bytes > MAX_TABLE_BYTES) return MINDIST_CPU_E_NOMEM;
    for (int l = 1; l <= s; ++l) {
        Level *v = &L[l];
        v->n = binom(k, l);
        v->sum = (uint64_t *)malloc(sizeof(uint64_t) * W * (v->n ? v->n : 1));
        v->last = (uint8_t *)malloc(v->n ? v->n : 1);
        if (!v->sum || !v->last) return MINDIST_CPU_E_NOMEM;
        uint64_t i = 0;
        for (int x = 0; x < k; ++x) {
            if (l == 1) {
                memcpy(v->sum + i * W, R + (size_t)x * W, sizeof(uint64_t) * W);
                v->last[i] = (uint8_t)x;
                ++i;
                continue;
            }
            const Level *u = &L[l - 1];
            const uint64_t from = u->n - binom(k - x - 1, l - 1);
            for (uint64_t j = from; j < u->n; ++j, ++i) {
                xor_into(v->sum + i * W, R + (size_t)x * W, u->sum + j * W, W);
                v->last[i] = u->last[j];
            }
        }
    }
    return 0;
}

/* index of the first lexicographic l-subset whose first element is >= f */
static inline uint64_t first_from(int k, int l, int f) { return binom(k, l) - binom(k - f, l); }

typedef struct {
    const Level *L;
    int k, W, s, r, off, unroll;
} Saved;

/* the last chunk (r rows) against one prefix, or two prefixes at once */
static void last_chunk(const Saved *q, const uint64_t *p1, int from1, const uint64_t *p2, int from2,
                       int with_prefix, Acc *a) {
    const Level *v = &q->L[q->r];
    const int W = q->W;
    uint64_t i1 = first_from(q->k, q->r, from1);
    if (p2) {
        /* entries from from1 on serve p1 only until from2, then both */
        const uint64_t i2 = first_from(q->k, q->r, from2);
        for (; i1 < i2; ++i1) {
            uint64_t x[MAXW];
            xor_into(x, p1, v->sum + i1 * W, W);
            const int wt = q->off + weight_of(x, W);
            if (wt < a->min) a->min = wt;
            ++a->combos;
            ++a->adds;
        }
        for (uint64_t i = i2; i < v->n; ++i) {
            const uint64_t *e = v->sum + i * W;
            uint64_t x[MAXW], y[MAXW];
            xor_into(x, p1, e, W);
            xor_into(y, p2, e, W);
            const int w1 = q->off + weight_of(x, W), w2 = q->off + weight_of(y, W);
            if (w1 < a->min) a->min = w1;
            if (w2 < a->min) a->min = w2;
        }
        a->combos += 2 * (v->n - i2);
        a->adds += 2 * (v->n - i2);
        return;
    }
    for (uint64_t i = i1; i < v->n; ++i) {
        int wt;
        if (with_prefix) {
            uint64_t x[MAXW];
            xor_into(x, p1, v->sum + i * W, W);
            wt = q->off + weight_of(x, W);
        } else {
            wt = q->off + weight_of(v->sum + i * W, W);
        }
        if (wt < a->min) a->min = wt;
    }
    a->combos += v->n - i1;
    if (with_prefix) a->adds += v->n - i1;
}

/* chunks t..: prefix holds the sum of the chunks before, `from` the first
 * element the next chunk may use, `left` the rows still to choose */
static void saved_step(const Saved *q, const uint64_t *prefix, int from, int left, int with_prefix,
                       Acc *a) {
    if (left == q->r) {
        last_chunk(q, prefix, from, NULL, 0, with_prefix, a);
        return;
    }
    const Level *v = &q->L[q->s];
    const int W = q->W;
    const int after = left - q->s;          /* rows after this chunk */
    uint64_t pending = UINT64_MAX;          /* unroll: a valid entry waiting for a partner */
    uint64_t pend_sum[MAXW];
    for (uint64_t i = first_from(q->k, q->s, from); i < v->n; ++i) {
        if ((int)v->last[i] + after >= q->k) continue;   /* no room for the rest */
        uint64_t np[MAXW];
        if (with_prefix) {
            xor_into(np, prefix, v->sum + i * W, W);
            ++a->adds;
        } else {
            memcpy(np, v->sum + i * W, sizeof(uint64_t) * W);
        }
        if (q->unroll && after == q->r) {
            if (pending == UINT64_MAX) {
                pending = i;
                memcpy(pend_sum, np, sizeof(uint64_t) * W);
                continue;
            }
            /* two prefixes: the one with the smaller last element has the
             * longer range of final chunks */
            const int f1 = v->last[pending] + 1, f2 = v->last[i] + 1;
            if (f1 <= f2) last_chunk(q, pend_sum, f1, np, f2, 1, a);
            else last_chunk(q, np, f2, pend_sum, f1, 1, a);
            pending = UINT64_MAX;
            continue;
        }
        saved_step(q, np, v->last[i] + 1, after, 1, a);
    }
    if (pending != UINT64_MAX) last_chunk(q, pend_sum, v->last[pending] + 1, NULL, 0, 1, a);
}

static int run_saved(const uint64_t *R, int k, int W, int w, int off, int s, int unroll, int nt,
                     Acc *out, double *table_seconds) {
    Level L[9];
    memset(L, 0, sizeof(L));
    const int ls = s < w ? s : w;
    const double t0 = omp_get_wtime();
    int rc = build_levels(R, k, W, ls, L);
    if (table_seconds) *table_seconds = omp_get_wtime() - t0;
    if (rc == 0) {
        Saved q = {L, k, W, ls, w - ls * ((w - 1) / ls), off, unroll};
        if (w <= ls) {
            Acc a = {INT32_MAX, 0, 0};
            last_chunk(&q, NULL, 0, NULL, 0, 0, &a);
            merge(out, &a);
        } else {
            const Level *v = &L[ls];
            const int after = w - ls;
#pragma omp parallel num_threads(nt)
            {
                Acc a = {INT32_MAX, 0, 0};
                /* the first chunk's entries, a few at a time, dynamically */
#pragma omp for schedule(dynamic, 64)
                for (int64_t i = 0; i < (int64_t)v->n; ++i) {
                    if (unroll && after == q.r) {
                        /* entries 2t and 2t+1 in one iteration, sharing the
                         * reads of the last chunk when both have room */
                        if (i & 1) continue;
                        const uint64_t j = (uint64_t)i + 1;
                        const int ok1 = (int)v->last[i] + after < k;
                        const int ok2 = j < v->n && (int)v->last[j] + after < k;
                        if (ok1 && ok2) {
                            const int f1 = v->last[i] + 1, f2 = v->last[j] + 1;
                            if (f1 <= f2) last_chunk(&q, v->sum + i * W, f1, v->sum + j * W, f2, 1, &a);
                            else last_chunk(&q, v->sum + j * W, f2, v->sum + i * W, f1, 1, &a);
                        } else if (ok1) {
                            last_chunk(&q, v->sum + i * W, v->last[i] + 1, NULL, 0, 1, &a);
                        } else if (ok2) {
                            last_chunk(&q, v->sum + j * W, v->last[j] + 1, NULL, 0, 1, &a);
                        }
                        continue;
                    }
                    if ((int)v->last[i] + after >= k) continue;   /* no room for the rest */
                    saved_step(&q, v->sum + (uint64_t)i * W, v->last[i] + 1, after, 1, &a);
                }
#pragma omp critical
                merge(out, &a);
            }
        }
    }
    for (int l = 1; l <= 8; ++l) {
        free(L[l].sum);
        free(L[l].last);
    }
    return rc;
}

int mindist_cpu_pair(const uint64_t *rows, int k, int words, int w, int offset, int algorithm,
                     int s, int threads, int32_t *pair_min, uint64_t *combinations,
                     uint64_t *additions, double *table_seconds) {
    if (!rows || !pair_min || k < 1 || k > MAXG || words < 1 || words > MAXW || w < 1 || w > k ||
        algorithm < MINDIST_CPU_BASIC || algorithm > MINDIST_CPU_SAVED_UNROLL2)
        return MINDIST_CPU_E_ARG;
    if (algorithm >= MINDIST_CPU_SAVED && (s < 1 || s > 8)) return MINDIST_CPU_E_ARG;
    const int nt = threads > 0 ? threads : omp_get_max_threads();
    if (table_seconds) *table_seconds = 0;
    Acc out = {INT32_MAX, 0, 0};
    int rc = 0;
    switch (algorithm) {
        case MINDIST_CPU_BASIC:
            run_basic(rows, k, words, w, offset, nt, &out);
            break;
        case MINDIST_CPU_OPTIMIZED:
        case MINDIST_CPU_STACK:
            if (w == 1) {
                /* no prefix: every row on its own */
                for (int e = 0; e < k; ++e) {
                    const int wt = offset + weight_of(rows + (size_t)e * words, words);
                    if (wt < out.min) out.min = wt;
                }
                out.combos = (uint64_t)k;
            } else {
                run_optimized(rows, k, words, w, offset, algorithm == MINDIST_CPU_STACK, nt, &out);
            }
            break;
        default:
            rc = run_saved(rows, k, words, w, offset, s, algorithm == MINDIST_CPU_SAVED_UNROLL2, nt, &out,
                           table_seconds);
    }
    if (rc) return rc;
    *pair_min = out.min;
    if (combinations) *combinations = out.combos;
    if (additions) *additions = out.adds;
    return 0;
}
