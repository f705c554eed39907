/*
 * mindist.h -- C ABI of the MI355X (gfx950) minimum-distance library.
 *
 * The library computes the minimum distance d of a binary linear code with
 * the Brouwer-Zimmerman method as described by Hernando, Igual and
 * Quintana-Orti, "Fast Algorithms for the Computation of the Minimum
 * Distance of a Random Linear Code": Section 2 (definition of d, information
 * sets, systematic matrices Gamma_j, Algorithm 1 with its upper bound U and
 * lower bound L) and Section 3 (enumerating every g-subset of the rows of a
 * Gamma_j with few row additions; Algorithm 5's left/right split with saved
 * right sums is the scheme the GPU kernel follows).
 *
 * Conventions for every entry point:
 *   - a matrix G is k rows of W = ceil(n/64) uint64 words, row-major; column
 *     c is bit (c % 64) of word (c / 64); bits >= n must be zero;
 *   - 1 <= k < n <= 512 (Section 2 assumes n > k);
 *   - all pointers are host pointers unless stated; inputs are copied, the
 *     caller keeps ownership of everything it passes;
 *   - return value 0 on success, a negative MINDIST_E_* code otherwise; no
 *     exception crosses the ABI; mindist_last_error() gives a per-thread
 *     message for the last failure;
 *   - a context is not thread-safe; separate contexts are independent.
 *
 * Process-wide state besides the per-thread error text (all of it
 * mutex-guarded, safe to use from several threads):
 *   - caches of device memory, pinned host memory, streams and events that
 *     contexts, batches and servers take from and return to, so that a run
 *     allocates nothing after warm-up; they grow to the largest working set
 *     seen and are released when the process ends;
 *   - per device: the binomial table C(x, t) (x <= 512, t <= 64) and the
 *     chunk-group tables of the pair shapes met so far (a few KB each), both
 *     read-only once uploaded;
 *   - per device, only once mindist_run_noalloc has run there: its static
 *     buffer of MINDIST_NOALLOC_BYTES and a lock.
 * The library assumes one HIP runtime in the process: a caller passing
 * streams from another framework (PyTorch ships its own HIP runtime) must
 * load that framework's runtime first, so the library binds to it.
 */
#ifndef MINDIST_H
#define MINDIST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MINDIST_OK            0
#define MINDIST_E_ARG        -1   /* null pointer, n/k out of range, nonzero padding bits */
#define MINDIST_E_RANK       -2   /* rank(G) < k */
#define MINDIST_E_NOMEM      -3   /* host or device allocation failed */
#define MINDIST_E_HIP        -4   /* HIP runtime error (no device, launch failure, ...) */
#define MINDIST_E_LIMIT      -5   /* a pair whose C(k,w) exceeds 2^63, or level > 64 */
#define MINDIST_E_CANCELLED  -6   /* stopped by MINDIST_OPT_CANCEL_AFTER_CHUNKS */
#define MINDIST_E_TIMEOUT    -7   /* MINDIST_OPT_DEADLINE_MS elapsed */
#define MINDIST_E_STATE      -8   /* call out of order (e.g. results before a run) */
#define MINDIST_E_CERT       -9   /* the result failed its certificate (mindist_certify):
                                     the visited pairs, their counts or bounds differ from
                                     Algorithm 1's, a pair stopped early although the least
                                     weight found was above the bound before it, or the
                                     witness is not a codeword of weight d */

#define MINDIST_MAX_N      512
#define MINDIST_MAX_WORDS  8
#define MINDIST_MAX_LEVEL  64

/* ---- options (mindist_set_option keys) ------------------------------- */
/* Termination granularity.  Algorithm 1 raises L once per level; Section 2
 * notes it may be raised after every Gamma_j.  0 = after every Gamma_j
 * (default), 1 = once per level (literal Algorithm 1). */
#define MINDIST_OPT_TERM             1
/* 1 (default) = stop a pair as soon as U <= L before that pair (only with
 * per-pair termination); the visited pairs, d and every pair minimum are
 * unchanged, only the executed count of the final pair shrinks. */
#define MINDIST_OPT_MIDPAIR_EXIT     2
/* The partial (rank k_m < k) information set, Algorithm 1's loop over
 * j = 1..m with Section 2's bound term f_m(g) = max(0, g+1-(k-k_m)):
 * 0 (default) = enumerate it at every level, as the loop does;
 * 1 = drop it and its bound term;
 * 2 = only when useful: from the first level g0 = k-k_m at which its term is
 *     positive.  The term counts only once every level up to g is done under
 *     Gamma_m, so at g0 the set also enumerates its levels 1..g0-1
 *     (ascending, after the full sets' pairs of level g0); later levels visit
 *     it once, at their own level.  d is the same under all three; the
 *     visited pairs differ. */
#define MINDIST_OPT_PARTIAL          3
/* 1 = also accumulate the sum of weights of every pair (checkable against a
 * closed form); slower.  0 (default) off. */
#define MINDIST_OPT_VERIFY           4
/* HIP stream (hipStream_t cast to int64) for all device work of this
 * context; 0 = a private stream created by the library (default). */
#define MINDIST_OPT_STREAM           5
/* wall-clock limit of one run in ms; 0 = none.  Checked between pairs. */
#define MINDIST_OPT_DEADLINE_MS      6
/* kernel shape: right-table entries per chunk; 0 (default) = chosen per
 * pair: the shortest tile (16..256) whose chunks fit one round of the
 * resident waves, else the longest (128..1024) that leaves every wave at
 * least max(2, D-1) chunks (D = 32-bit words per codeword). */
#define MINDIST_OPT_TILE_T           7
/* kernel shape: resident workgroups per CU the enumeration launches are
 * sized for; 0 (default) = 4, or for the matrix-core kernel (MINDIST_OPT_MFMA)
 * as many as its registers let one CU hold, at most 4 (2 at 3 and 4 words
 * with 4 lane items). */
#define MINDIST_OPT_BLOCKS_PER_CU    8
/* 1 = time every enumeration launch with HIP events (seconds_enum). */
#define MINDIST_OPT_PROFILE          9
/* testing: stop with MINDIST_E_CANCELLED once this many chunks of the run
 * have been claimed; 0 = off. */
#define MINDIST_OPT_CANCEL_AFTER_CHUNKS 10
/* cap on the saved right-sum table of one (Gamma_j, size) in MiB
 * (default 1024). */
#define MINDIST_OPT_TABLE_MIB        11
/* kernel shape: left subsets held per lane in one chunk (2 or 4, default 4). */
#define MINDIST_OPT_LANE_ITEMS       12
/* 1 (default) = read left subsets from a saved table when it fits the
 * table cap; 0 = every lane unranks its left subsets and adds their rows. */
#define MINDIST_OPT_LEFT_TABLES      13
/* chunk order within a pair: 0 (default) = left-tile-major, 1 =
 * right-tile-major (the resident waves share the same few right tiles). */
#define MINDIST_OPT_CHUNK_ORDER      14
/* chunk dispensers per pair: 8 (default) interleaved counters, or 1. */
#define MINDIST_OPT_COUNTERS         15
/* kernel shape: left subsets a pair's split should provide so that one
 * pair keeps every resident wave busy; the split moves rows from the right
 * to the left side (shorter right runs, at least 64 entries) until it does.
 * 0 = always the balanced split. */
#define MINDIST_OPT_MIN_ITEMS        16
/* launching ahead: the next pair is launched right behind the current one,
 * before that one's result is read, so the device never waits for the host
 * between pairs.  0 = off; any other value: with mid-pair exit on (the
 * default) and no deadline every next pair is launched ahead -- if
 * Algorithm 1 stops before it, its waves read U <= its bound and leave at
 * once, and it is not reported; otherwise only a pair of at most this many
 * combinations is (it would run to its end), default 2^28.  Never when the
 * bound after the current pair reaches the Singleton bound, nor with a
 * chunk budget. */
#define MINDIST_OPT_SPECULATE        17
/* testing: seed the device's least weight found with this value (and no
 * witness) before the first pair; 0 (default) = off.  A value below the true
 * distance makes the kernels stop a pair early (they see U <= L before it)
 * while the host's U, the least pair minimum, is higher: the run must fail
 * with MINDIST_E_CERT instead of returning a result whose enumeration
 * stopped short.  A value above the true distance changes nothing. */
#define MINDIST_OPT_INJECT_U         18
/* inner loop of the two-level pairs of at most 4 words per codeword (the
 * weights are the same either way): 1 (default) = the part of a chunk that
 * every lane subset covers, in whole blocks of 32 right entries, on the
 * int8 matrix cores (wt(l ^ r) = wt(l) + sum_k r_k (1 - 2 l_k), one
 * 32 x 32 x 32 product per word); 0 = XOR and popcount on the vector ALUs
 * throughout.  VERIFY runs always use the vector ALUs.  Single-code path
 * only: the batch and serving kernel always runs such pairs on the matrix
 * cores. */
#define MINDIST_OPT_MFMA             19

typedef struct mindist_ctx mindist_ctx;

typedef struct mindist_result {
    int32_t  d;               /* minimum distance (Algorithm 1's returned U) */
    int32_t  n, k;
    int32_t  m_full;          /* number of disjoint full-rank information sets */
    int32_t  k_partial;       /* rank of the partial set (0 if none) */
    int32_t  n_gamma;         /* Gamma matrices enumerated (m_full [+1]) */
    int32_t  w_last, j_last;  /* last visited pair (level w, set j, 0-based j) */
    int32_t  L_final;         /* lower bound when the run stopped */
    int32_t  U_found;         /* least weight found (n+1 if none) */
    int32_t  pairs_visited;
    int32_t  exited_midpair;  /* 1 if the last pair was cut short */
    int32_t  witness_j, witness_w;   /* pair of the witness */
    uint64_t witness[MINDIST_MAX_WORDS];       /* codeword of weight d, layout of G */
    uint64_t witness_rows[MINDIST_MAX_WORDS];  /* bit r set = row r of Gamma_{witness_j} used */
    uint64_t executed_total;  /* codewords evaluated on the GPU */
    uint64_t canonical_total; /* sum of C(k,w) over visited pairs */
    double   seconds_total;   /* wall clock of mindist_run (host preprocessing is in create) */
    double   seconds_enum;    /* summed enumeration-kernel time (HIP events, PROFILE=1) */
    int32_t  enum_launches;   /* enumeration kernel launches in this run */
    int32_t  reserved;
} mindist_result;

/* one visited pair (Algorithm 1, one iteration of the inner loop) */
typedef struct mindist_pair {
    int32_t  j, w;            /* set index (0-based, partial set last) and level */
    int32_t  L_before, L_after, U_after;
    int32_t  pair_min;        /* least weight over the pair */
    uint64_t count;           /* C(k,w): combinations the pair covers */
    uint64_t executed;        /* combinations evaluated (< count only if cut short) */
    uint64_t wsum;            /* sum of weights (VERIFY=1 only, else 0) */
    double   ms;              /* kernel time of the pair's launch (PROFILE=1 only) */
    int32_t  dwords;          /* 32-bit words carried per codeword by the kernel */
    int32_t  split_a;         /* rows per lane subset */
    int32_t  split_b;         /* rows from the (outer) right table */
    int32_t  split_b2;        /* rows from the inner table (0: two-level split) */
    int32_t  launch;          /* single path: index of the first pair of the launch this pair
                                 ran in (short consecutive pairs share one launch; 0 in batch
                                 and serving records) */
    double   t_start_ms;      /* PROFILE=1: when the pair's kernel started, ms after the first
                                 pair's; batch and serving: when the pair's job opened, ms after
                                 the code's first job opened (ms is then the open-to-close time) */
    double   dev_ms;          /* single path, always: the pair's part of its enumeration launch
                                 on the device clock, from its first wave's start to its last
                                 wave's end (no dispatch latency); 0 in batch and serving */
} mindist_pair;

/* Section 2 and Algorithm 1 preprocessing: validate and copy G, greedy
 * disjoint information sets over the columns in ascending order, the
 * reduced echelon Gamma_j of each set, and the device copies the
 * enumeration needs.  Needs a HIP device.  *out is owned by the caller and
 * released with mindist_destroy. */
int mindist_create(const uint64_t *G, int n, int k, mindist_ctx **out);

/* set an option (MINDIST_OPT_*) before mindist_run */
int mindist_set_option(mindist_ctx *ctx, int key, int64_t value);

/* partition summary of a created context */
int mindist_info(const mindist_ctx *ctx, int *m_full, int *k_partial, int *n_gamma);

/* Algorithm 1: raise the level until L >= U.  Blocking.  `out` is caller-
 * owned.  May be called again (results are recomputed from scratch). */
int mindist_run(mindist_ctx *ctx, mindist_result *out);

/* the visited pairs of the last run, in visiting order */
int mindist_get_pairs(const mindist_ctx *ctx, mindist_pair *out, int cap, int *n_out);

/* NULL-safe */
void mindist_destroy(mindist_ctx *ctx);

const char *mindist_last_error(void);

/* For callers that cannot allocate device or pinned memory (work between
 * HIP graph captures, tight serving loops, harnesses that forbid hipMalloc):
 * mindist_create + mindist_run + mindist_destroy of one code in a single
 * call that allocates no device or pinned memory.  Its device state (run
 * state, mailboxes, per-wave totals, chunk groups, Gamma_j rows and the
 * saved-sum tables of the pair being enumerated) lives in one static device
 * buffer of MINDIST_NOALLOC_BYTES per GPU, reserved the first time the call
 * runs on that GPU and held until the process ends.  Default options
 * (per-pair termination, mid-pair exit, partial set at every level); pairs
 * run one at a time (none launched ahead), lanes unrank their left subsets,
 * and a set's table level is capped so one table's levels fit a quarter of
 * the buffer's table arena (about 23 MiB): d, the visited pairs, their
 * bounds, minima and counts equal mindist_run's, timings differ.
 * G, n, k as in mindist_create; stream: hipStream_t cast to int64, 0 = the
 * null stream; out: caller-owned result; pairs: optional caller-owned array
 * of pairs_cap records receiving the visited pairs (*n_pairs = how many were
 * visited, even beyond pairs_cap; n_pairs may be NULL).  Blocking: the
 * stream is idle on return.  Calls on one GPU share its buffer and run one
 * at a time (a lock per GPU; each call clears what it needs); a call that
 * overlapped another on the same GPU without that lock would race.
 * Errors: as mindist_create / mindist_run, MINDIST_E_LIMIT if a code needs
 * more of the buffer than it holds (not reached for n <= 512 on a GPU with
 * at most 256 compute units). */
#define MINDIST_NOALLOC_BYTES (96u << 20)
int mindist_run_noalloc(const uint64_t *G, int n, int k, int64_t stream, mindist_result *out,
                        mindist_pair *pairs, int pairs_cap, int *n_pairs);

/* Calibration microbenchmark: the enumeration kernel's inner loop (one
 * 32-bit XOR + popcount per carried word and a min per codeword, right sums
 * from scalar loads) over registers and a 64-entry table, on every CU, with
 * no setup, tails or atomics.  Reports codewords/s for `dwords` carried
 * words per codeword (1, 2, 3, 4, 7 or 8).  A reference for the instruction
 * mix, not a ceiling: on gfx950 the enumeration kernel itself runs 5-10 %
 * faster (its right runs are longer than the table walked here). */
int mindist_calibrate(int dwords, int blocks_per_cu, double *codewords_per_s, double *seconds);

/* The measured ceiling of the enumeration's arithmetic on this GPU: a
 * register-only kernel on every compute unit (blocks_per_cu blocks of 256
 * lanes, 1..16) whose loop is nothing but 32-bit XOR + popcount pairs
 * (v_xor_b32 with a wave-uniform operand that changes every step,
 * v_bcnt_u32_b32 accumulating) over words held in registers, in independent
 * chains per lane; no memory operation in the loop.  variant 0..3 sets
 * (chains per lane, words per chain, steps per loop iteration) = (8, 4, 1),
 * (8, 4, 4), (4, 6, 4), (16, 2, 4).  Writes the best of three timed launches
 * (after one warm-up) as 32-bit XOR+popcount operations per second (one per
 * lane per word) and its duration; seconds may be NULL.  Blocking.  The
 * best over variants and occupancies is the denominator of the kernels'
 * VALU roofline where it exceeds the figure derived from the rated clock. */
int mindist_peak_xorpop(int variant, int blocks_per_cu, double *ops_per_s, double *seconds);

/* Comparison kernel for one pair (Gamma_j, w) of a created context (Section
 * 3.3, the stack-based enumeration of Algorithm 4, as a GPU walk): every
 * lane unranks its own start in lexicographic order (combinatorial number
 * system) and walks consecutive w-subsets, the last element moving fastest
 * over rows held in LDS, one row addition per codeword plus the partial
 * sums rebuilt at each carry.  It only measures that direct walk against
 * the saved-sums kernel that mindist_run uses; it changes no state of the
 * context.  j indexes the enumerated sets (full sets in order, then the
 * partial set), 1 <= w <= 12, k <= 128 and at most 4 carried 32-bit words
 * per row (n - k <= 128 for a full set, n <= 128 for the partial set), else
 * MINDIST_E_LIMIT.  blocks_per_cu 0 = 4 (at most 16).  Outputs: the least
 * weight of the pair, the combinations evaluated (C(k, w)) and the kernel
 * time from HIP events; executed and seconds may be NULL.  Blocking. */
int mindist_walk_pair(mindist_ctx *ctx, int j, int w, int blocks_per_cu, int32_t *pair_min,
                      uint64_t *executed, double *seconds);

/* The current HIP device: its architecture name (e.g. "gfx950", written to
 * name with at most cap bytes including the terminator) and its compute
 * unit count.  Either output may be NULL. */
int mindist_device(char *name, int cap, int *compute_units);

/* Host-only planning (no device needed): the greedy partition and the
 * systematic matrices.  sets: n ints (full sets of k columns each, then the
 * partial set); gammas: n_gamma * k * W words (full sets first, partial last;
 * pass NULL to skip).  Returns MINDIST_OK or an error. */
int mindist_plan(const uint64_t *G, int n, int k, int *sets, int *m_full,
                 int *k_partial, uint64_t *gammas);

/* Host-only: the lower bound after pair (j, w) under per-Gamma termination
 * (Section 2): sum over sets i <= j of f_i(w) plus over i > j of f_i(w-1),
 * f_full(h) = h+1, f_partial(h) = max(0, h+1-(k-k_m)). */
int mindist_bound_after(int k, int m_full, int k_partial, int include_partial,
                        int j, int w);

/* Host-only: Algorithm 1's pair order (Section 2) for a partition with
 * m_full >= 1 full sets and a partial set of rank k_partial (0 = none) under
 * MINDIST_OPT_PARTIAL's policy (0, 1, 2) and termination rule (per_level 0 =
 * raise L after every Gamma_j, 1 = once per level), up to level k, as if no
 * codeword were ever found.  Pair t is written to out[4t .. 4t+3] = (set j,
 * level w it enumerates, Algorithm 1's outer level g, L after it); at most
 * cap pairs are written and *n_out receives the schedule's length.  Errors:
 * MINDIST_E_ARG. */
int mindist_schedule(int k, int m_full, int k_partial, int partial_policy, int per_level,
                     int32_t *out, int cap, int *n_out);

/* the run a certificate checks: the code's size and partition and the
 * options it ran under */
typedef struct mindist_cert_spec {
    int32_t n, k, m_full, k_partial;
    int32_t partial_policy;   /* MINDIST_OPT_PARTIAL */
    int32_t per_level;        /* MINDIST_OPT_TERM */
    int32_t midpair_exit;     /* MINDIST_OPT_MIDPAIR_EXIT */
} mindist_cert_spec;

/* Host-only: the certificate every run of mindist_run, mindist_run_batch and
 * the servers passes before it returns a result (Section 2, Algorithm 1's
 * termination; the run returns MINDIST_E_CERT otherwise).  The visited pairs
 * must follow mindist_schedule's order from L = 1 and U = n-k+1; each covers
 * C(k, w) combinations and every completed one evaluated exactly that many;
 * L_before, L_after and U_after of each pair equal the recomputed values
 * (U = the least pair minimum so far, capped at n-k+1); Algorithm 1's test
 * L < U held before each pair (before each level under per_level); only the
 * last pair may be cut short, only with mid-pair exit, and only when U <= L
 * before it; the run ended because L >= U, because its last pair was cut,
 * or because level k was done; d equals the final U and L_final the final L;
 * exited_midpair says whether the last pair was cut.  Only the fields j, w,
 * L_before, L_after, U_after, pair_min, count and executed of pairs are
 * read.  Returns MINDIST_OK, MINDIST_E_CERT (reason in mindist_last_error)
 * or MINDIST_E_ARG. */
int mindist_certify(const mindist_cert_spec *spec, const mindist_pair *pairs, int n_pairs,
                    int d, int L_final, int exited_midpair);

/* Host-only: the r-subset {x_1 < ... < x_r} of [0, hi) whose colex rank
 * sum_t C(x_t, t) is `rank` (the combinatorial number system the kernels
 * and the witness decoding use), written to out[0..r) ascending.
 * 0 <= r <= 64, r <= hi <= 512, rank < C(hi, r); else MINDIST_E_ARG. */
int mindist_colex_unrank(uint64_t rank, int r, int hi, int *out);

/* ---- batches: many codes in one persistent launch ---------------------- */
typedef struct mindist_batch_opts {
    int32_t tile_min;         /* right-tile length bounds (0 = 2048 / 4096; the maximum is raised
                                 to the minimum if below it) */
    int32_t tile_max;
    int32_t blocks_per_cu;    /* resident workgroups per CU (0 = 4; capped at what the
                                 persistent kernel's registers allow: 2) */
    int32_t use_graph;        /* 1 = run as one captured hipGraph (default), 0 = plain launch */
    int32_t table_kib;        /* cap on one saved right-sum table in KiB (0 = 65536) */
    int32_t jobs_per_code;    /* job-arena sizing: average jobs per code (0 = 96) */
    int32_t chunks_per_visit; /* chunks a wave runs on one code's job before it moves on to
                                 the next code with work (0 = 4; -1 = until the job is fully
                                 claimed): the share of waves each live code gets; a job of
                                 1024 chunks or more is always run until fully claimed */
    int32_t direct_log2;      /* routing: a code expected to enumerate at least 2^direct_log2
                                 combinations (estimate: every pair while the bound is below a
                                 Gilbert-Varshamov estimate of d), or beyond the persistent
                                 kernel's limits, runs through the single-code path on one of
                                 8 worker threads (own streams, side by side) after the
                                 persistent launch; 0 = 30; -1 = every code in the persistent
                                 launch (the tuning knobs above apply to that launch only) */
    double  deadline_s;       /* wall-clock limit of the call; waves leave after it and the
                                 call returns MINDIST_E_TIMEOUT (0 = none) */
    int64_t stream;           /* hipStream_t, 0 = private */
    mindist_pair *pairs;      /* optional: visited pairs of every code (caller-owned) */
    int64_t pairs_cap;        /* capacity of pairs[] */
    int64_t *pairs_index;     /* optional: B+1 offsets into pairs[] (caller-owned) */
    double  seconds_kernel;   /* out: device time of the persistent launch (HIP events) plus
                                 the wall time of the codes run through the single path */
    double  seconds_total;    /* out: wall clock of the call */
    double  seconds_prep;     /* out: host preprocessing (information sets, packing) */
    uint64_t executed_total;  /* out: codewords evaluated */
    /* out: profile of the launch, summed over its waves: seconds spent in
     * table chunks, in enumeration chunks and in job completion (flushes and
     * the opening of the next job); the rest of waves * seconds_kernel is
     * spent looking for work */
    double  wave_s_table, wave_s_pair, wave_s_flush;
    int64_t waves;            /* out: waves of the launch */
    uint64_t chunks_table, chunks_pair;   /* out: chunks run of each kind */
    double  *done_s;          /* optional, caller-owned, B entries: seconds from the first
                                 code's start on the device to code i's completion (-1 if
                                 it did not run) */
} mindist_batch_opts;

/* Solve B codes in one persistent launch: a device-side scheduler hands out
 * chunks of each code's current pair (Algorithm 1's inner minimum) and, when a
 * pair completes, applies Algorithm 1's bound and termination test for that
 * code and opens its next pair (one raise of L per Gamma_j, midpair exit).
 * Codes expected to be long (see direct_log2) run through the single-code
 * path instead, on worker threads after the launch.  G[i] points at code
 * i's matrix (layout as above; in the persistent launch rows of at most 256
 * carried bits (n <= 256 when there is a partial set), k <= 256 and at most
 * 32 information sets, other codes are routed to the single path unless
 * direct_log2 = -1); out has B caller-owned entries.  Results equal
 * mindist_run's with default options (d, visited pairs, counts, pair minima);
 * witnesses may differ but have weight d.  Per-code failures (rank, limits)
 * are reported as out[i].d = negative error code; the call returns
 * MINDIST_OK unless the whole batch failed. */
int mindist_run_batch(const uint64_t *const *G, const int *n, const int *k, int B,
                      mindist_result *out, mindist_batch_opts *opts);

/* ---- serving: continuous batching of arriving codes ---------------------
 *
 * Codes submitted to a server wait in a queue and are admitted, in
 * submission order among those that fit, as slots and device memory free
 * up; their work overlaps on the device with the codes already running.
 *
 * Engine 0 (default): max_active worker threads, each running one admitted
 * code at a time through the single-code path (mindist_create / run /
 * destroy) on its own stream; the device runs the kernels of all codes in
 * flight side by side.  Engine 1: one stream and a set of code slots on the
 * device; a manager thread keeps the persistent multi-code kernel of
 * mindist_run_batch running over the resident codes; to admit waiting
 * codes the launch is stopped (every wave finishes the chunk it holds, so
 * no work is lost), the new codes' slots are written and the kernel is
 * launched again over old and new codes together; a code's information
 * sets, Gamma_j, saved tables, bounds and job records stay on the device
 * from admission to completion, and finished codes are read back while the
 * others keep running.
 *
 * Under either engine a code's result equals mindist_run's with default
 * options (d, visited pairs, counts, pair minima); witnesses may differ but
 * have weight d. */
typedef struct mindist_server mindist_server;

typedef struct mindist_server_opts {
    int32_t max_active;       /* codes running at once: engine 0, worker threads (0 = 8);
                                 engine 1, code slots resident on the device (0 = 256) */
    int32_t blocks_per_cu;    /* engine 1: resident workgroups per CU of the persistent kernel
                                 (0 = as many as its registers allow, 2; 1 while it routes
                                 codes to the single path, leaving half of each SIMD's
                                 registers to their kernels) */
    int64_t device_bytes;     /* device memory for the codes in flight: a code is admitted
                                 only when its share fits beside theirs (0 = 8 GiB).  Engine
                                 0: estimated rows, saved right and left tables up to half
                                 the expected top level, run state; engine 1: rows,
                                 saved tables and witness slots in a pool allocated at
                                 creation (routed codes use the single path's own memory).
                                 Submit fails with MINDIST_E_NOMEM for a code whose share
                                 exceeds it */
    double  epoch_min_ms;     /* engine 1: least running time of a launch before it is
                                 stopped so that waiting codes that cannot be admitted
                                 into it come in (0 = 0.5 ms) */
    int32_t table_kib;        /* cap on one saved table in KiB (0 = the single-code path's
                                 1 GiB for engine 0, 65536 for engine 1) */
    int32_t jobs_per_code;    /* job records per slot (0 = 96); a code needing more ends
                                 with MINDIST_E_LIMIT */
    int32_t chunks_per_visit; /* as in mindist_batch_opts (0 = 4) */
    int32_t engine;           /* 0 (default): each admitted code runs the single-code path
                                 (mindist_create / run / destroy) on its own stream in one of
                                 max_active worker threads; the device runs the kernels of
                                 the codes in flight side by side.  1: the persistent
                                 multi-code kernel, admitting codes while it runs (epoch_min_ms, jobs_per_code,
                                 blocks_per_cu, chunks_per_visit and linger_ms apply to this
                                 engine only) */
    double  linger_ms;        /* engine 1: how long a launch with no code left keeps running
                                 for the next arrivals (0 = 200 ms, negative = it ends at
                                 once); its idle waves sleep between looks */
    int32_t route_log2;       /* engine 1: codes expected to enumerate at least
                                 2^route_log2 combinations run through the single-code
                                 path on 4 worker threads beside the persistent kernel,
                                 which then holds 2 blocks per CU unless blocks_per_cu says
                                 otherwise (0 = 2^24; -1 = none, every code in the kernel) */
} mindist_server_opts;

#define MINDIST_SERVER_MAX_PAIRS 256

typedef struct mindist_server_result {
    uint64_t tag;             /* the caller's tag from submit */
    int32_t  status;          /* MINDIST_OK or a negative MINDIST_E_* */
    int32_t  n_pairs;         /* entries of pairs[] */
    mindist_result result;
    double   t_submit, t_admit, t_done;   /* seconds on the server clock */
    mindist_pair pairs[MINDIST_SERVER_MAX_PAIRS];   /* visited pairs, in order */
} mindist_server_result;

typedef struct mindist_server_stats {
    uint64_t submitted, admitted, completed;
    uint64_t epochs;          /* launches of the persistent kernel (engine 1): a launch runs
                                 while codes are resident and admits arriving ones; it is
                                 stopped when a waiting code needs a relaunch to come in
                                 (every free slot already used in it, pool ranges freed in
                                 it, rows beyond 32 KiB), when no code has been left for
                                 linger_ms, after 20 ms while routed codes are in flight,
                                 and after 10 s */
    double   seconds_kernel;  /* engine 1: summed launch time (HIP events); engine 0: summed
                                 enumeration kernel time of the finished codes (device clock) */
    int32_t  resident;        /* codes being run now (engine 1: on the device or routed) */
    int32_t  pending;         /* codes waiting for admission now */
    uint64_t admitted_live;   /* engine 1: codes admitted into a running launch (the rest of
                                 `admitted` were written between launches or routed) */
    uint64_t routed;          /* engine 1: codes run through the single path (route_log2) */
} mindist_server_stats;

/* Start a server on the current HIP device (opts may be NULL).  *out is
 * released with mindist_server_destroy. */
int mindist_server_create(const mindist_server_opts *opts, mindist_server **out);
/* Validate and copy G (layout as in mindist_create), compute its
 * information sets and Gamma_j on the calling thread, and queue it.
 * Returns at once with MINDIST_OK, or the error of that preprocessing
 * (nothing is queued then).  Thread-safe. */
int mindist_server_submit(mindist_server *s, const uint64_t *G, int n, int k, uint64_t tag);
/* Non-blocking: move up to cap finished results (caller-owned array) to
 * out, oldest first; *n_out receives their number.  Thread-safe. */
int mindist_server_poll(mindist_server *s, mindist_server_result *out, int cap, int *n_out);
/* Block until no code is waiting or resident, or timeout_s seconds passed
 * (MINDIST_E_TIMEOUT); results stay queued for poll. */
int mindist_server_wait(mindist_server *s, double timeout_s);
/* seconds since the server started (the clock of t_submit/t_admit/t_done) */
double mindist_server_clock(const mindist_server *s);
int mindist_server_stats_get(const mindist_server *s, mindist_server_stats *out);
/* Engine 1: stop the kernel and the manager thread; unfinished codes are
 * dropped.  Engine 0: waiting codes are dropped, codes being run finish
 * first, then the workers end.  NULL-safe. */
void mindist_server_destroy(mindist_server *s);

#ifdef __cplusplus
}
#endif
#endif /* MINDIST_H */
