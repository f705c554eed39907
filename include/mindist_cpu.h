/* mindist_cpu.h -- the paper's CPU enumeration algorithms (Section 3) as
 * measured host baselines: one pair (Gamma, w) = all w-subsets of the k rows
 * of a systematic matrix, their sums and least weight.  Built as its own
 * library (libmindist_cpu.so) from plain C with OpenMP; the GPU library
 * never calls it.
 *
 * Rows: k rows of `words` uint64 words each (the columns the weight counts,
 * packed as in mindist.h); weight of a combination = offset + popcount of
 * the XOR of its rows.  Additions are counted as whole-row XORs, the unit of
 * the section's cost lemmas.
 *
 * Errors: MINDIST_CPU_E_ARG (-1) for NULL pointers, k outside 1..256, words
 * outside 1..8, w outside 1..k, an unknown algorithm, s outside 1..8 for
 * the saved algorithms; MINDIST_CPU_E_NOMEM (-3) when the saved tables
 * (C(k,l) entries for l <= s) cannot be allocated. */
#ifndef MINDIST_CPU_H
#define MINDIST_CPU_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MINDIST_CPU_E_ARG    -1
#define MINDIST_CPU_E_NOMEM  -3

/* Algorithm 2: every combination in lexicographic order, its w rows added
 * from scratch (w - 1 additions per combination). */
#define MINDIST_CPU_BASIC          0
/* Algorithm 3: the (w-1)-combinations in lexicographic order, their sum
 * built from scratch and reused for every last element. */
#define MINDIST_CPU_OPTIMIZED      1
/* Algorithm 4: as Algorithm 3, with a stack of partial sums rebuilt only
 * from the leftmost element that changed. */
#define MINDIST_CPU_STACK          2
/* Algorithm 5: saved sums of all l-subsets, l <= s, in lexicographic order;
 * a combination is split into chunks of s rows (the last chunk 1..s rows)
 * read from the saved levels, floor((w-1)/s) additions per combination. */
#define MINDIST_CPU_SAVED          3
/* Section 3.5: Algorithm 5 with two prefixes processed against each saved
 * entry of the last chunk (each entry read once for both). */
#define MINDIST_CPU_SAVED_UNROLL2  4

/* One pair with `threads` OpenMP threads (0 = the OpenMP default), dynamic schedule over
 * the outermost loop (Section 4's parallelisation).  Outputs: least weight,
 * combinations evaluated (C(k, w)), row additions, and for the saved
 * algorithms the time spent building the saved levels (built on every call;
 * the section builds them once per Gamma); all but pair_min may be NULL.
 * Returns 0 or a negative error. */
int mindist_cpu_pair(const uint64_t *rows, int k, int words, int w, int offset, int algorithm,
                     int s, int threads, int32_t *pair_min, uint64_t *combinations,
                     uint64_t *additions, double *table_seconds);

#ifdef __cplusplus
}
#endif
#endif
