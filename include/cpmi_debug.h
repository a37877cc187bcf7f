/*
 * cpmi_debug.h -- diagnostic entry points of the cpmi library, used by the
 * test-suite to check device behaviour the public calls depend on. Same
 * conventions as cpmi.h (device pointers owned by the caller, synchronous).
 */
#ifndef CPMI_DEBUG_H
#define CPMI_DEBUG_H

#include <stdint.h>

#include "cpmi.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One 32x32 matrix-core product through the screen's fragment path:
 * C[r][c] = sum_k A[r][k] * B[c][k] over one 32-byte K slice per row.
 * A, B: device, 32 rows x 32 bytes (FP32: 8 values, BF16: 16, int8: 32 per
 * row); C: device float [32][32]. precision: CPMI_PREC_F32, _BF16 or _I8.
 * Checks the operand/accumulator lane layouts the screen assumes. */
int cpmi_dbg_mfma_probe(int precision, const void *A, const void *B, float *C, void *stream);

/* The sustained matrix-core rate of device `device` in TFLOP/s (TOP/s for
 * int8): one work-group per compute unit, each wave issuing 16 independent
 * 32x32 accumulations (CPMI_PREC_F32, _BF16 or _I8 operands, the screen's
 * instructions) for `iters` rounds from registers, timed with HIP events.
 * *ms_out (host, nullable): the timed launch. Allocates and frees its own
 * output buffer; synchronises the device's null stream. Returns the rate, or
 * a negative CPMI_ERR_* code. */
double cpmi_dbg_mfma_peak(int device, int precision, int iters, double *ms_out);

/* The screen bound on the hardware. Runs the builder and the real screen
 * kernel (tile edge `tile`, 128 or 256, at `precision`) over the m tiles
 * tiles_ij (host int64 [m][2], block row I and block column J of edge tile),
 * and writes every element's screen value D~ (row I*tile + il, column
 * J*tile + jl) to dump_out (device, m*tile*tile, row-major per tile; float,
 * or int32 for int8), its canonical d2 computed by the verifier to d2_out
 * (device double, same indexing; elements whose row or column is past the
 * last row are not written), each tile's bound E (the applied per-tile bound
 * of the screen) to bound_out (host double [m]) and the largest
 * |D~ - d2| / E over the tiles' elements to *max_ratio_out (host; for int8 0
 * when every value is exact, else infinity). src: device points (series = 0:
 * n x d rows of stride ld, float32 or int8) or a float32 series of length n
 * whose z-normalised windows of length d are the rows (series = 1). The
 * bound is what makes the screen exact; a ratio above 1 would break it.
 * Errors: ERR_ARG (shapes, a tile out of range), ERR_NONFINITE,
 * ERR_DEGENERATE, ERR_RANGE, ERR_HIP. */
int cpmi_dbg_screen_sample(cpmi_ctx *ctx, const void *src, int dtype, int64_t n, int64_t d, int64_t ld, int series,
                           int precision, int tile, const int64_t *tiles_ij, int64_t m, void *dump_out,
                           double *d2_out, double *bound_out, double *max_ratio_out, void *stream);

/* Run only the l-mer builder on a series and return the canonical window
 * means and sigmas (device double [len - ell + 1] each), so that they can be
 * compared bit for bit with the definition (Section 2 windows, two-pass
 * population z-normalisation). */
int cpmi_dbg_znorm(cpmi_ctx *ctx, const float *series, int64_t len, int64_t ell, int precision, double *mu,
                   double *sigma, void *stream);

/* Host only (no device work): the screen's tile list for one problem of n
 * rows with exclusion excl and tile edge `tile` (128 or 256). Entries are
 * packed as problem << 44 | I << 22 | J (block row, block column); unused
 * slots are all ones. Writes min(count, cap) entries to out (host) and returns
 * the count, or ERR_ARG. */
int64_t cpmi_dbg_tile_list(int64_t n, int64_t excl, int tile, uint64_t *out, int64_t cap);

/* Host only: the tile list of a two-set problem (the string searches of
 * cpmi_strings_pair with CPMI_LEAST_CORRELATED and of cpmi_two_locus): na
 * rows of the first set, nb of the second starting at row split (a multiple
 * of 256, >= na); a pair (i, j) is admissible iff i < na, split <= j <
 * split + nb and j - split != i. Writes min(count, cap) entries to out and
 * the number of leading full-tile slots to *nfull (nullable); returns the
 * count, or ERR_ARG. */
int64_t cpmi_dbg_tile_list_two(int64_t na, int64_t nb, int64_t split, int tile, uint64_t *out, int64_t cap,
                               int64_t *nfull);

/* Host only: the screening-error bound applied to every pair of a tile whose
 * row blocks have maxima bI, bJ = (s^, ||x||, ||x~||, ||x - x~||) (4 floats
 * each), padded dimension kpad, true dimension d, screen precision, and
 * screen value form: 0 = row scalars added after the product (128-row
 * screen), 1 = row scalars folded into the product (256-row screen). */
double cpmi_dbg_tile_bound(const float *bI, const float *bJ, int32_t kpad, int64_t d, int precision, int form);

/* Host only: the 256-tile screen's K-slice layout for direct-to-LDS load
 * (wave 0..3, block q 0..3, lane 0..63): out4 = {tile row read, byte column
 * read within the 64-byte slice, LDS byte written, LDS byte at which a
 * fragment read of that (row, chunk) looks}. */
int cpmi_dbg_layout256(int wave, int q, int lane, int32_t *out4);

/* Host only: byte offset of byte `byte` of row `row` in the screen operand
 * of the 256-row screen (rows of `rowbytes` bytes, a multiple of 128),
 * which is stored slice-major per block of 256 rows; -1 for bad arguments. */
int64_t cpmi_dbg_xs_offset256(int64_t row, int64_t byte, int64_t rowbytes);

/* Copy `bytes` (a multiple of 16) from src to dst (device, non-overlapping)
 * with a plain vector copy kernel: a launch of known traffic (bytes read,
 * bytes written) against which the hardware byte counters are scaled. */
int cpmi_dbg_copy(void *dst, const void *src, int64_t bytes, void *stream);

/* Host only: the lower bound that reference-point pruning applies to every
 * pair of a tile whose row blocks have, for each of q references, distance
 * intervals [loI[k], hiI[k]] and [loJ[k], hiJ[k]] (host arrays of q
 * doubles): max over k of the gap between the intervals, less a margin for
 * the rounding of the distances (Section 3, triangle inequality). */
double cpmi_dbg_tile_lb(const double *loI, const double *hiI, const double *loJ, const double *hiJ, int q);

/* Host only: the tile list of the reference-point pruned search of one point
 * set of n rows (tile edge 128 or 256, q references): lo, hi (host, nT * q
 * doubles, nT = ceil(n / tile)) are the per-block distance intervals, block
 * I's interval for reference k at [I * q + k] (any order of the blocks; the
 * enumeration stops early where reference 0's intervals allow). A tile (I, J), I <= J,
 * is kept unless some reference's intervals, each widened by 2^-34 |hi|,
 * are more than T apart (T < 0: every tile dropped); band >= 0 keeps only
 * J - I <= band. Writes min(count, cap) entries (packed as
 * cpmi_dbg_tile_list) to out, the leading full-tile slots to *nfull and the
 * tiles dropped to *npruned (both nullable); returns the count, or ERR_ARG. */
int64_t cpmi_dbg_pruned_tiles(int64_t n, int tile, int q, const double *lo, const double *hi, double T, int64_t band,
                              uint64_t *out, int64_t cap, int64_t *nfull, int64_t *npruned);

/* The same list built by the library's device kernels (the list the pruned
 * searches screen): lo, hi host arrays as above, copied to the device; tiles
 * in bands of 8 block rows; exclusion excl (1 for point sets); permuted != 0
 * for windows in reference order (every tile partial). Entries and counts as
 * cpmi_dbg_pruned_tiles with band = -1 (out: host). Synchronises `stream`.
 * Returns the count, or ERR_ARG / ERR_HIP. */
int64_t cpmi_dbg_pruned_tiles_gpu(cpmi_ctx *ctx, int64_t n, int tile, int q, const double *lo, const double *hi,
                                  double T, int64_t excl, int permuted, uint64_t *out, int64_t cap, int64_t *nfull,
                                  int64_t *npruned, void *stream);

/* Row order of the pruned radius searches with two or more references:
 * order 0 (default) sorts the rows by buckets of width w * R of their
 * distance to the first reference and by their distance to the second within
 * a bucket; order 1 by the first reference alone (as closest-pair queries
 * always do). w > 0 (default 1). Returns CPMI_OK or ERR_ARG. */
int cpmi_dbg_set_prune_order(cpmi_ctx *ctx, int order, double w);

/* Host only: the tuning decisions of a context with `ncu` compute units
 * after reading the cache file cache_in (nullable): the precision and tile a
 * call with (dtype, precision, d, pairs) would use, as cpmi_tune_lookup. If
 * cache_out is not NULL the loaded cache is written there as
 * cpmi_save_tune_cache would. */
int cpmi_dbg_tune(const char *cache_in, const char *cache_out, int ncu, int dtype, int precision, int64_t d,
                  double pairs, int32_t *prec_out, int32_t *tile_out);

#ifdef __cplusplus
}
#endif

#endif /* CPMI_DEBUG_H */
