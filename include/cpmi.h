/*
 * cpmi.h -- exact closest pair, fixed-radius neighbours and time-series motifs
 * on AMD Instinct MI355X (gfx950).
 *
 * Problems (Rajasekaran & Pathak, "Efficient Algorithms for the Closest Pair
 * Problem and Applications", 2014):
 *   - closest pair (CPP, Section 3): given n points in R^d, the pair at least
 *     Euclidean distance (distance as defined in Section 2);
 *   - fixed-radius near neighbours (FRNNP, Section 3.5): for every point, the
 *     other points within distance R; returned here as the canonical list of
 *     pairs i<j with d(i,j) <= R, from which N(i) is the symmetric closure;
 *   - time-series motif (Section 2 l-mers, Section 3 problem statement): the two
 *     closest l-mers of a series T. Windows are z-normalised and a pair of
 *     windows (i, j) is admissible only if j - i >= excl (overlapping windows
 *     are trivial matches);
 *   - the most and the least correlated pair of strings over a small alphabet
 *     (Sections 4-5; correlation = fraction of agreeing positions), exactly
 *     through the one-hot encoding on the INT8 matrix cores, or by the
 *     randomised light-bulb bucketing (MLBA);
 *   - the two-locus association pair of SNPs (Section 6).
 *
 * Reference-point pruning (MPR, Section 3) can be switched on for the point
 * and single-series motif searches (cpmi_set_pruning).
 *
 * Every answer is exact with respect to the canonical FP64 arithmetic below,
 * whatever the screening precision: a Gram-form screen on the matrix cores
 * (FP32, BF16 or INT8) is followed by an FP64 re-verification of every pair
 * whose screening error interval can reach the current minimum or the radius.
 *
 *   Canonical squared distance of rows x, y (float input): x_k, y_k promoted to
 *   double; acc = 0; for k = 0..d-1: t = x_k - y_k; acc = fma(t, t, acc).
 *   int8 input: sum_k (x_k - y_k)^2 in integers (exact).
 *   z-normalisation of window i (length l): mu = (sum_{k ascending} T[i+k]) / l,
 *   v = (sum_{k ascending} fma(e, e, .), e = T[i+k] - mu) / l (population
 *   variance), sigma = sqrt(v), xhat_k = (T[i+k] - mu) / sigma, all in double.
 *   Ties in the closest pair go to the lexicographically smallest (i, j).
 *
 * Conventions for every call:
 *   - Indices are 0-based (the paper's are 1-based).
 *   - Input arrays (points, series) and output arrays named "device" are device
 *     pointers owned by the caller (for example from torch.empty(device="cuda")).
 *     The library never frees or retains them after the call returns.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL is the null stream) and
 *     the call returns after the stream has finished the work it enqueued;
 *     results in host structs and device arrays are then valid.
 *   - A context is not thread-safe; use one context per host thread.
 *   - Return value: CPMI_OK (0) or a negative CPMI_ERR_* code; the message is
 *     available from cpmi_last_error(ctx). No exception crosses this ABI.
 */
#ifndef CPMI_H
#define CPMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cpmi_ctx cpmi_ctx;

/* return codes */
enum {
    CPMI_OK = 0,
    CPMI_ERR_ARG = -1,        /* invalid argument (shape, stride, dtype, precision, NULL pointer) */
    CPMI_ERR_NOPAIR = -2,     /* no admissible pair (n < 2, or len < ell + excl for a motif)       */
    CPMI_ERR_NONFINITE = -3,  /* the input holds NaN or Inf                                         */
    CPMI_ERR_DEGENERATE = -4, /* a window has zero variance, so it cannot be z-normalised           */
    CPMI_ERR_CAPACITY = -5,   /* the caller's output array is too small; *count_out holds the need  */
    CPMI_ERR_HIP = -6,        /* a HIP runtime call failed                                          */
    CPMI_ERR_RANGE = -7       /* a squared norm is too large for the FP32 screen (>= 2^100)         */
};

/* element type of the input points */
enum { CPMI_F32 = 0, CPMI_I8 = 1 };

/* screening precision; every precision returns the same exact answer */
enum {
    CPMI_PREC_AUTO = 0, /* the tuned choice for the shape (INT8 for int8 input)          */
    CPMI_PREC_F32 = 1,  /* FP32 matrix-core screen (plain form)                          */
    CPMI_PREC_BF16 = 2, /* BF16 operands, FP32 accumulation, rigorous per-tile bound     */
    CPMI_PREC_I8 = 3    /* int8 operands, int32 accumulation: exact, no bound needed     */
};

/* Result of a closest-pair search. d2 is the canonical squared distance and d
 * its correctly rounded square root. screen_err is the largest |screen value -
 * d2| over the candidates that were re-verified, and screen_bound the largest
 * error bound that was applied to them (screen_err <= screen_bound always;
 * both 0 for int8). status is CPMI_OK or the per-item error code. */
typedef struct {
    int64_t i, j;
    double d2;
    double d;
    double screen_err;
    double screen_bound;
    int32_t status;
    int32_t reserved;
} cpmi_pair;

/* Statistics of the last call on a context. */
typedef struct {
    int64_t valid_pairs;         /* admissible pairs of the problem                           */
    int64_t tiles_total;         /* screen tiles evaluated in the first pass                  */
    int64_t tiles_rescreened;    /* tiles whose lower bound reached the minimum (second pass) */
    int64_t cpp_candidates;      /* pairs re-verified in FP64 for the closest pair            */
    int64_t frnn_candidates;     /* pairs re-verified in FP64 for the radius                  */
    int64_t frnn_pairs;          /* pairs within the radius                                   */
    int64_t reruns;              /* internal buffer growths that forced a re-run              */
    double max_err_over_bound;   /* max over verified candidates of |screen - d2| / bound      */
    double kernel_ms;            /* device time of the enqueued work, HIP events              */
    double screen_ms;            /* device time of the main first-pass screen launch (HIP
                                    events on the call's stream; 0 when replayed from a graph) */
    int64_t screen_pairs;        /* admissible pairs covered by that launch                    */
    int32_t precision;           /* precision actually used (CPMI_PREC_*)                     */
    int32_t tile;                /* screen tile edge used                                     */
    int64_t tiles_pruned;        /* tiles dropped by the reference-point bound (cpmi_set_pruning) */
} cpmi_stats;

/* Create a context on HIP device `device`. tune_cache_path (nullable) names a
 * JSON file of tuned screen configurations written by cpmi_save_tune_cache; if
 * NULL or unreadable the built-in defaults are used. *out: host. Errors:
 * ERR_ARG (out NULL, no such device), ERR_HIP (the HIP runtime could not
 * enumerate devices or create the context's stream and events). */
int cpmi_create(cpmi_ctx **out, int device, const char *tune_cache_path);

/* Release the context and its device workspace. NULL is accepted. */
int cpmi_destroy(cpmi_ctx *ctx);

/* Closest pair of n points (Section 3 problem statement; MPR step 5 keeps the
 * least distance). pts: device, row-major n x d with row stride ld elements
 * (ld >= d), dtype CPMI_F32 or CPMI_I8. out: host. Errors: ERR_ARG (n, d, ld,
 * dtype, precision), ERR_NOPAIR (n < 2), ERR_NONFINITE, ERR_RANGE. */
int cpmi_closest_pair(cpmi_ctx *ctx, const void *pts, int dtype, int64_t n, int64_t d, int64_t ld,
                      int precision, void *stream, cpmi_pair *out);

/* Closest pair as cpmi_closest_pair, without allocating: for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc). Every device buffer of the search is a
 * slice of a static device array of CPMI_NOALLOC_SCRATCH_BYTES per GPU, which
 * the library holds until the process ends; no hipMalloc, hipFree or pinned
 * host allocation is made (results come back through pageable host memory).
 * Same arguments, layout, result and errors as cpmi_closest_pair, plus
 * ERR_CAPACITY when the search does not fit the array: the screen operand
 * (n rounded up to 256 rows of d rounded up to the screen's K step, 2 bytes
 * per element in BF16, 4 in FP32, 1 in int8), the row scalars, the tile lists
 * and room for at least 1024 closest-pair candidates (e.g. up to about 40,000
 * BF16 points of d = 512), or when more than 2^20 candidates tie within the
 * screening bound. The reference-point pruning switch is ignored. All calls on
 * one GPU share its array: calls that overlap in time on one GPU (several
 * threads or streams) race and give undefined results; serialise them. */
#define CPMI_NOALLOC_SCRATCH_BYTES (64ull << 20)
int cpmi_closest_pair_noalloc(cpmi_ctx *ctx, const void *pts, int dtype, int64_t n, int64_t d, int64_t ld,
                              int precision, void *stream, cpmi_pair *out);

/* Fixed-radius pairs (Section 3.5, MPR-FRNNS emits j into N(i) and i into N(j)
 * when d <= R): every pair i<j with canonical d2 <= R2, sorted by (i, j).
 * R2 is the squared radius (callers pass fl(R*R); for int8 data an integer).
 * pairs: device int64 [cap][2] (may be NULL when cap == 0); d2: device
 * double [cap] or NULL; count_out: host. If the count exceeds cap, nothing is
 * written to pairs/d2, *count_out holds the count and ERR_CAPACITY is
 * returned (call again with cap >= count). The count is exact at any size
 * (64-bit, also beyond 2^32 pairs); one call returns at most 2^28 pairs: above
 * that, or when more than 2^28 pairs lie within the screening bound of R2
 * (the pairs are then counted, not stored), ERR_CAPACITY is returned with the
 * exact count whatever cap is. */
int cpmi_frnn(cpmi_ctx *ctx, const void *pts, int dtype, int64_t n, int64_t d, int64_t ld, double R2,
              int precision, void *stream, int64_t *pairs, double *d2, int64_t cap, int64_t *count_out);

/* Closest pair and fixed-radius pairs of the same points from one screening
 * pass. best (host) may be NULL to skip the closest pair; R2 < 0 skips the
 * radius search (pairs, d2, count_out may then be NULL). Same errors as above. */
int cpmi_points(cpmi_ctx *ctx, const void *pts, int dtype, int64_t n, int64_t d, int64_t ld,
                int precision, double R2, void *stream, cpmi_pair *best,
                int64_t *pairs, double *d2, int64_t cap, int64_t *count_out);

/* Neighbour lists N(i) of a radius search (Section 3.5: MPR-FRNNS outputs,
 * for every point i, the other points within R) as compressed rows. pairs:
 * device int64 [m][2], distinct pairs (i, j) with 0 <= i < j < n, in any
 * order (as cpmi_frnn, cpmi_points and cpmi_motif return them); row_ptr:
 * device int64 [n + 1]; cols: device int64 [2m]. The neighbours of point v
 * are cols[row_ptr[v] .. row_ptr[v + 1]), ascending; every pair appears under
 * both of its points. Buffers are the caller's; the library's workspace grows
 * by about 32 (m + n) bytes. Synchronises `stream`. Errors: ERR_ARG (n < 1,
 * n >= 2^31, m < 0, m >= 2^31, a NULL buffer that is needed, or a pair outside
 * 0 <= i < j < n: row_ptr and cols are then unspecified), ERR_HIP. */
int cpmi_pairs_to_csr(cpmi_ctx *ctx, const int64_t *pairs, int64_t m, int64_t n, int64_t *row_ptr, int64_t *cols,
                      void *stream);

/* Motif of a series (Section 3: the two closest l-mers of T). series: device
 * float32 [len]; windows i = 0..len-ell are z-normalised; pairs with
 * j - i < excl are excluded (excl <= 0 means excl = ell). best: host (may be
 * NULL to skip). If R2 >= 0, all admissible window pairs with d2 <= R2 are also
 * returned as for cpmi_frnn. Errors: ERR_ARG (ell < 2, len < ell),
 * ERR_NOPAIR (len - ell + 1 <= excl), ERR_NONFINITE, ERR_DEGENERATE. */
int cpmi_motif(cpmi_ctx *ctx, const float *series, int64_t len, int64_t ell, int64_t excl,
               int precision, double R2, void *stream, cpmi_pair *best,
               int64_t *pairs, double *d2, int64_t cap, int64_t *count_out);

/* Motifs of many series in one batched launch sequence (one persistent screen
 * over the tiles of all series, replayed from a captured HIP graph when the
 * same shapes are seen again). series: host array of nseries device pointers
 * to float32 series; lens, ells: host arrays; exclusion is ell per series.
 * best: host [nseries]; best[s].status carries the per-series error code
 * (ERR_NOPAIR, ERR_NONFINITE, ERR_DEGENERATE) while the call returns CPMI_OK
 * if the arguments were valid. */
int cpmi_motif_batch(cpmi_ctx *ctx, const float *const *series, const int64_t *lens, const int64_t *ells,
                     int64_t nseries, int precision, void *stream, cpmi_pair *best);

/* Message describing the last error on ctx (empty string if none). Valid until
 * the next call on ctx. */
const char *cpmi_last_error(cpmi_ctx *ctx);

/* Copy the statistics of the last successful call into *out. */
int cpmi_last_stats(cpmi_ctx *ctx, cpmi_stats *out);

/* Set the screen configuration used by later calls with `precision` (tile edge
 * 128 or 256 for the matrix-core screen); 0 restores the default. Used by the
 * autotuner. Returns ERR_ARG for an unsupported value. */
int cpmi_set_tile(cpmi_ctx *ctx, int precision, int tile);

/* Autotuner result: the fastest precision tried and its fastest tile edge,
 * and the best device time (ms, HIP events around the whole call) of every
 * configuration tried, indexed [precision][tile 128, tile 256]; 0 where not
 * tried. For the 256 tile also the band height of the tile order chosen
 * (block rows per band; 0 if the 128 tile won) and the times of bands 4, 8
 * and 16, indexed [precision][band]. */
typedef struct {
    int32_t precision;
    int32_t tile;
    double ms[4][2];
    int32_t band;
    int32_t reserved;
    double band_ms[4][3];
} cpmi_tune_result;

/* Autotuner: time a closest-pair search (the screen configurations the
 * library has: tile edge 128 or 256; with CPMI_PREC_AUTO on float32 input
 * also FP32 against BF16 screening; for the 256 tile the band height of the
 * tile order, 4, 8 or 16 block rows) on the caller's points, `reps` timed calls
 * after one warm-up each, and record in the context the fastest tile and band
 * for each precision tried and, for AUTO, the fastest precision, keyed by
 * precision, dimension bucket (next power of two >= max(d, 64)) and size
 * bucket (ceil(log2) of the row count of a point set with as many pairs).
 * Later calls on problems in the same buckets use these choices; batched
 * motifs use the precision and tile of the bucket of their largest l and of
 * their total pair count, and each series the band of its own l and pair
 * count. Arguments as
 * for cpmi_closest_pair; out: host. Errors: as cpmi_closest_pair, ERR_ARG for
 * reps outside 1..1000. */
int cpmi_autotune(cpmi_ctx *ctx, const void *pts, int dtype, int64_t n, int64_t d, int64_t ld, int precision,
                  void *stream, int reps, cpmi_tune_result *out);

/* Write every tuned choice of the context as the JSON object that
 * cpmi_create reads ({"bf16:k512:r18": 256, "auto:k512:r18": 2,
 * "band.bf16:k512:r18": 8, ...}; the "auto" value is a CPMI_PREC_* code, a
 * "band." entry a band height). The file is replaced atomically.
 * Errors: ERR_ARG if the file cannot be written. */
int cpmi_save_tune_cache(cpmi_ctx *ctx, const char *path);

/* The precision and tile a call would use for float32 (CPMI_F32) or int8
 * input of dimension d with `pairs` admissible pairs under `precision`
 * (after tuning, the cache, or the built-in rule: tile 256 when the problem
 * has at least four 256x256 tiles per compute unit, else 128). prec_out,
 * tile_out: host. Does not touch the GPU. */
int cpmi_tune_lookup(cpmi_ctx *ctx, int dtype, int precision, int64_t d, double pairs, int32_t *prec_out,
                     int32_t *tile_out);

/* The band height of the tile order (block rows per band of the 256-tile
 * screen) a problem of dimension d with `pairs` admissible pairs uses at
 * `precision` (CPMI_PREC_F32, _BF16 or _I8): tuned (or from the cache), else
 * 8. In a batched motif call each series uses its own. band_out: host. Does
 * not touch the GPU. */
int cpmi_tune_lookup_band(cpmi_ctx *ctx, int precision, int64_t d, double pairs, int32_t *band_out);

/* Reference-point tile pruning (MPR, Section 3: reference points projected
 * by a factor f, points ordered by their distance to the first reference,
 * pairs dropped when the triangle-inequality lower bound exceeds the current
 * upper bound). With q >= 1 the point calls (cpmi_closest_pair, cpmi_frnn,
 * cpmi_points) and the single-series motif call (cpmi_motif, on the
 * z-normalised windows) pick q reference rows (windows) from `seed`, project
 * them by f (every coordinate times f), order the rows by their distance to
 * the first projected reference, and skip every screen tile whose rows are
 * provably farther apart than both the least distance found between
 * neighbouring blocks in that order and the radius. A pruned motif always
 * uses the 256-row screen, which applies the exclusion zone to the window
 * positions of the reordered rows. Answers are unchanged (exact);
 * stats.tiles_pruned counts the skipped tiles. q = 0 turns it off (the
 * default). cpmi_motif_batch is never pruned. Errors: ERR_ARG for q outside
 * 0..32 or f not finite and > 0. */
int cpmi_set_pruning(cpmi_ctx *ctx, int q, double f, uint64_t seed);

/* Result of a string-pair search. i < j are the two strings (SNPs for
 * cpmi_two_locus); matches counts the positions where they agree
 * (cpmi_strings_pair: u_ij of Section 5; cpmi_two_locus: the matching bits of
 * columns i and n + j of D), out of `length` (k, or the column length
 * 3 (m1 + m2)). status as in cpmi_pair. */
typedef struct {
    int64_t i, j;
    int64_t matches;
    int64_t length;
    int32_t status;
    int32_t reserved;
} cpmi_match_pair;

/* modes of cpmi_strings_pair */
enum { CPMI_MOST_CORRELATED = 0, CPMI_LEAST_CORRELATED = 1 };

/* Most or least correlated pair of n strings of length k over the alphabet
 * {0, ..., sigma-1} (Section 5: the correlation of two strings is the fraction
 * of positions where they agree, so the most correlated pair is the closest
 * pair in Hamming distance). strings: device, int8, row i = string i, row
 * stride ld >= k. Computed exactly and by brute force on the INT8 matrix
 * cores through the one-hot encoding of Section 5 (each symbol -> sigma bits
 * with one set): the squared distance of two code rows is their Hamming
 * distance 2 (k - u_ij), and between a code row and a complemented one it is
 * sigma k - 2 (k - u_ij) (the identity M(A'_i, ~A'_j) = 2 (k - u_ij)), so the
 * least correlated pair is the closest (code, complement) pair with i != j.
 * Ties go to the lexicographically smallest (i, j). out: host. Needs n >= 2,
 * k >= 1, 2 <= sigma <= 64, sigma k <= 2^20. Errors: ERR_ARG (shapes, mode,
 * or a symbol outside the alphabet), ERR_NOPAIR (n < 2). */
int cpmi_strings_pair(cpmi_ctx *ctx, const int8_t *strings, int64_t n, int64_t k, int64_t ld, int sigma,
                      int mode, void *stream, cpmi_match_pair *out);

/* Randomised light-bulb bucketing (Section 4, MLBA; Section 5 for the least
 * correlated pair), a candidate generator for the problem of
 * cpmi_strings_pair. Each of `iterations` iterations picks `columns` random
 * columns (distinct; drawn from `seed`), sorts the rows by their values in
 * those columns, and adds every pair of rows with equal values there (one
 * bucket) to the candidates; each candidate's exact match count is computed
 * and the best pair kept (ties to the lexicographically smallest (i, j)).
 * CPMI_MOST_CORRELATED buckets the strings themselves (columns are
 * positions, at most 64 / ceil(log2 sigma) of them); CPMI_LEAST_CORRELATED
 * buckets the one-hot codes against their complements (columns are bit
 * positions of the codes, at most 64; bit c sigma + b is set where symbol c
 * is sigma - 1 - b, Section 5's order) and keeps (code, complement) pairs of
 * different strings. The answer is the exact best pair with high probability
 * only (enough iterations; the paper's analysis); the reported count is
 * always the pair's exact one. *pairs_out (host, nullable) receives the
 * number of candidate pairs collected over all iterations (the paper's
 * measure of work). cap: candidate pairs one iteration may hold. strings:
 * device, as for cpmi_strings_pair; out: host. Needs n < 2^21 - 1 and
 * k < 2^22. Errors:
 * ERR_ARG (shapes, mode, columns, iterations, cap, a symbol outside the
 * alphabet), ERR_NOPAIR (n < 2, or no two rows ever shared a bucket),
 * ERR_CAPACITY (an iteration produced more than cap candidates; *pairs_out
 * counts the pairs of the iterations run until then, that one included).
 * The columns of an iteration are the first `columns` entries of a partial
 * Fisher-Yates shuffle of 0..C-1 (C = k, or sigma k for the least correlated
 * pair), restarted from the identity for every iteration: step q swaps
 * entries q and q + (splitmix64(c) mod (C - q)), where c counts up from
 * seed * 0x9e3779b97f4a7c15 (mod 2^64) over the steps of all iterations and
 * splitmix64(c) is SplitMix64's output for state c (the state advanced by
 * 0x9e3779b97f4a7c15, then mixed). */
int cpmi_strings_lightbulb(cpmi_ctx *ctx, const int8_t *strings, int64_t n, int64_t k, int64_t ld, int sigma,
                           int mode, int iterations, int columns, uint64_t seed, int64_t cap, void *stream,
                           cpmi_match_pair *out, int64_t *pairs_out);

/* Two-locus association (Section 6): genotypes (device, int8 in {0, 1, 2},
 * (m1 + m2) x n, row s = subject s, row stride ld >= n; the first m1 rows
 * are cases, the rest controls). With A', B' the one-hot codes of the cases'
 * and controls' columns, returns the SNP pair (i, j), i != j, whose columns i
 * and n + j of D = [A' A'; B' ~B'] agree in the most bits (direction 0; that
 * count is m1 + 2 u_A(i,j) + 2 (m2 - u_B(i,j)), so the pair maximises
 * u_A - u_B, the number of subjects in which SNPs i and j agree among cases
 * minus among controls: P_A(i,j) - P_B(i,j) when m1 = m2), or of
 * D = [A' ~A'; B' B'] (direction 1: u_B - u_A). Exact, brute force on the
 * INT8 matrix cores; ties to the lexicographically smallest (i, j), reported
 * with i < j (the count is symmetric in i, j). out: host. Needs m1, m2 >= 1,
 * n >= 2, 3 (m1 + m2) <= 2^20. Errors: ERR_ARG (shapes, direction, or a value
 * outside {0, 1, 2}), ERR_NOPAIR (n < 2). */
int cpmi_two_locus(cpmi_ctx *ctx, const int8_t *genotypes, int64_t m1, int64_t m2, int64_t n, int64_t ld,
                   int direction, void *stream, cpmi_match_pair *out);

/* Library version (major * 10000 + minor * 100 + patch). */
int cpmi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CPMI_H */
