// Internal declarations shared by the host orchestration and the kernels of
// the cpmi library (not part of the public C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cpmi {

enum Prec : int { P_F32 = 1, P_BF16 = 2, P_I8 = 3 };

// Screen modes of the Gram kernel (bit set).
enum Mode : int {
    M_MIN = 1,   // pass 1: record the tile minimum of the screen value
    M_EMIT = 2,  // pass 2: emit pairs within the closest-pair and/or radius thresholds
    M_DUMP = 4   // test: write the screen value of every element of every listed tile
};

// One flag word per problem; set by the builders, read back by the host.
enum Flag : uint32_t { F_NONFINITE = 1u, F_DEGENERATE = 2u, F_RANGE = 4u, F_SYMBOL = 8u };

// A pair emitted by the screen: rows (i, j) of problem p and its screen value.
struct Cand {
    int32_t i, j;
    float dt;
    uint32_t p;
};

// Description of one problem (a point set, or the windows of one series).
struct Prob {
    const void *xs;        // screen operand: npad rows of kpad elements (FP32, BF16 bits or int8)
    const void *shat;      // npad row scalars: fp32(||x||^2), or the exact int32 ||x||^2 for int8
    const float4 *bmax;    // per block of `tile` rows: max of (s^, a, at, r), see bound.h
    const void *src;       // canonical data: float or int8 points, or the float series
    const double *mu;      // motif: canonical window means, else null
    const double *sigma;   // motif: canonical window sigmas, else null
    int64_t n;             // rows (points or windows)
    int64_t d;             // true dimension (point dimension or window length)
    int64_t ld;            // row stride of the point source (elements)
    int32_t kpad;          // padded dimension (elements) of xs rows
    int32_t excl;          // a pair is admissible iff j - i >= excl
    int32_t motif;         // 1 if the rows are z-normalised windows of src
    int32_t src_i8;        // 1 if src holds int8 points
    double r2;             // squared radius (negative: no radius search)
    int32_t form;          // screen value form of the screen used (SCREEN_EPILOGUE / SCREEN_FOLDED)
    int32_t split;         // two-set problem (int8, 256-row screen): first row of the second set, a
                           // multiple of 256; a pair (i < j) is admissible iff i < na, j >= split,
                           // j < n and j - split != i. 0 for a single set.
    const int32_t *perm;   // screen row r holds source row perm[r] (reference-point order), or null
    int64_t na;            // two-set problem: rows of the first set
    const uint2 *fold;     // BF16 screens: per row, fold_words(s^) (the folded row scalar), else null
    const float4 *rowstat; // radius searches (FP32 / BF16 screens): per screen row, that row's own
                           // (s^, a, at, r) of bound.h, else null
};

// The folded row scalar of the BF16 256-row screen: c = -s^/4 split into three
// BF16 parts c1 + c2 + c3 (each rounded to nearest even, the remainders exact),
// packed as (c1 | c2 << 16, c3 | 1.0 << 16) so that the screen builds its
// matrix-core operands [c1 c2 c3 1 1 1 0 0] / [1 1 1 c1 c2 c3 0 0] from two
// words. |c1 + c2 + c3 - c| <= 2^-27 |c|.
__host__ __device__ inline uint32_t bf16_rne_bits(float f)
{
    const uint32_t u = __builtin_bit_cast(uint32_t, f);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__host__ __device__ inline uint2 fold_words(float s)
{
    const float c = -0.25f * s;
    const uint32_t h1 = bf16_rne_bits(c);
    const float r1 = c - __builtin_bit_cast(float, h1 << 16);
    const uint32_t h2 = bf16_rne_bits(r1);
    const float r2 = r1 - __builtin_bit_cast(float, h2 << 16);
    const uint32_t h3 = bf16_rne_bits(r2);
    return make_uint2(h1 | (h2 << 16), h3 | (0x3f80u << 16));
}

// Source row of screen row r.
__host__ __device__ inline int64_t src_row(const Prob &P, int64_t r) { return P.perm ? (int64_t)P.perm[r] : r; }

// Tile-list entry: problem (20 bits) | block row I (22 bits) | block col J (22 bits).
__host__ __device__ inline uint64_t tile_pack(uint32_t p, uint32_t I, uint32_t J)
{
    return ((uint64_t)p << 44) | ((uint64_t)I << 22) | (uint64_t)J;
}
__host__ __device__ inline uint32_t tile_prob(uint64_t t) { return (uint32_t)(t >> 44); }
__host__ __device__ inline uint32_t tile_I(uint64_t t) { return (uint32_t)(t >> 22) & 0x3fffffu; }
__host__ __device__ inline uint32_t tile_J(uint64_t t) { return (uint32_t)t & 0x3fffffu; }
constexpr uint64_t TILE_NONE = ~0ull;

typedef unsigned long long u64c;   // 64-bit device counter (atomicAdd operand)

// Arguments of the Gram screen kernel.
struct ScreenArgs {
    const Prob *probs;
    const uint64_t *tiles;     // tile list
    int64_t ntiles;            // entries (pass 1); pass 2: entries of sel_dense
    const u64c *sel_count;     // pass 2: number of valid entries of `tiles` (below 2^31)
    // pass 2: the selected tiles in list order (TILE_NONE elsewhere, ntiles
    // entries), walked instead of `tiles` when more than a quarter of the
    // list is selected (it keeps the list's panel locality); or null
    const uint64_t *sel_dense;
    uint32_t *tile_min;        // pass 1: per entry, four words: each wave's min screen value (float or int32 bits)
    const double *U;           // pass 2: per problem closest-pair upper bound, or null (no pair search)
    Cand *candR;               // radius candidates
    u64c *cntR;                // their counter (may exceed capR: the required size)
    uint64_t capR;
    Cand *candU;               // closest-pair candidates
    u64c *cntU;
    uint64_t capU;
    // Counting form of the radius search (null: off). Pairs whose screen
    // value alone proves d^2 <= r2 (D~ <= r2 - bound) are only counted here;
    // the rest of the radius candidates (the band r2 - bound < D~ <= r2 +
    // bound) are emitted to candR as usual.
    u64c *cntIn;
    // M_DUMP: tile_edge^2 values per list entry, row-major within the tile
    // (float, or int32 for int8)
    void *dump;
    // 256 tile: some problem's rows hold 4k + 2 K slices of 64 bytes (else
    // every problem's a multiple of 4)
    bool k2;
};

// Wave-aggregated reservation of n slots per lane (called by every lane of
// the wave, in wave-uniform control flow): one atomic add per wave and
// counter. Returns this lane's first slot; lanes with n = 0 get an unused value.
__device__ inline uint64_t wave_reserve(u64c *cnt, uint32_t n)
{
    const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    uint32_t incl = n;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = (uint32_t)__shfl_up((int)incl, o, 64);
        if (lane >= o) incl += v;
    }
    const uint32_t total = (uint32_t)__shfl((int)incl, 63, 64);
    u64c base = 0;
    if (total != 0) {
        if (lane == 0) base = atomicAdd(cnt, (u64c)total);
        base = __shfl(base, 0, 64);
    }
    return (uint64_t)base + (incl - n);
}

// Sum of n over the wave added to *cnt with one atomic (same calling rules).
__device__ inline void wave_count(u64c *cnt, uint32_t n)
{
    uint32_t v = n;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
    const int lane = (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    if (lane == 0 && v != 0) atomicAdd(cnt, (u64c)v);
}

// Per-problem result of the verifier (device), reset before each run.
struct ResDev {
    unsigned long long best_d2;   // min canonical d2 over candidates (double bits; ~0 = none)
    unsigned long long best_ij;   // min (i << 32 | j) among candidates at best_d2
    unsigned int err_bits;        // max |screen - d2| over verified candidates (float bits, rounded up)
    unsigned int ratio_bits;      // max |screen - d2| / bound (float bits, rounded up)
    unsigned int bound_bits;      // max bound applied (float bits)
    unsigned int flags;           // F_* input flags of the problem
};

// Longest window of a series, and windows per builder block (which stages
// SERIES_WPB + ell - 1 values in LDS).
constexpr int SERIES_MAX_ELL = 8192;
constexpr int SERIES_WPB = 64;

// Job of the window builder: one series.
struct SeriesJob {
    const float *T;
    int64_t len;
    int64_t ell;
    int64_t npad;       // padded rows (windows) of xs
    int64_t blk_base;   // first builder block (SERIES_WPB windows) of this job (prefix sum)
    void *xs;
    void *shat;
    float4 *bmax;
    double *mu;
    double *sigma;
    unsigned int *flags;
    int32_t kpad;
    int32_t pad0;
    const int32_t *iperm;  // screen row of window w (reference order), or null for w itself
    uint2 *fold;           // BF16: per row fold_words(s^), else null
    float4 *rowstat;       // per-row bound terms (null: not written); with iperm they are also what
                           // launch_block_max reduces per block
};

// ---- launchers (defined in the .hip files) --------------------------------

// Fill n words with v (a kernel, so it is safe inside captured graphs).
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);
void launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t st);
void launch_reset_res(ResDev *r, int64_t n, hipStream_t st);
void launch_calib_copy(const void *src, void *dst, int64_t n16, hipStream_t st);

// Row preparation of points (float32 or int8): screen operand, row scalars,
// per-block maxima (bmax must be zero on entry), flags, and (float input,
// rowstat not null) each row's own bound terms.
void launch_prep_points(const void *pts, int dtype, int64_t n, int64_t d, int64_t ld, int prec, void *xs,
                        int32_t kpad, int64_t npad, void *shat, float4 *bmax, int tile, unsigned int *flags,
                        const int32_t *perm, uint2 *fold, float4 *rowstat, hipStream_t st);

// Window builder of many series: canonical mean/sigma, z-normalised screen
// operand, row scalars, block maxima (zero on entry), flags.
// bmax[b] = componentwise max of rowstat over the rows of block b (tile <= 256 rows).
void launch_block_max(const float4 *rowstat, int64_t npad, int tile, float4 *bmax, hipStream_t st);
void launch_prep_series(const SeriesJob *jobs, int64_t njobs, int64_t total_blocks, int prec, int tile,
                        hipStream_t st);

// Gram screen (grid = work-groups; pass 2 loops over *sel_count entries).
// masked = false promises that every pair of every listed tile is admissible
// (used by the 256-tile screen for its list of full tiles).
void launch_screen(int prec, int tile, int mode, bool masked, const ScreenArgs &a, int64_t grid, hipStream_t st);

// Pass 1 -> pass 2: U[p] = min over tiles of (tile min + bound); then the
// tiles whose lower bound (tile min - bound) does not exceed U[p] (if Ubits)
// or the problem's squared radius (if r2 >= 0).
void launch_reduce_U(const Prob *probs, const uint64_t *tiles, int64_t ntiles, const uint32_t *tile_min, int prec,
                     unsigned long long *Ubits, hipStream_t st);
void launch_select(const Prob *probs, const uint64_t *tiles, int64_t ntiles, const uint32_t *tile_min, int prec,
                   const unsigned long long *Ubits, uint64_t *sel, u64c *sel_count, uint64_t *dense, hipStream_t st);

// Candidate verification in canonical FP64 (exact int64 for int8).
void launch_verify_cpp(const Prob *probs, const Cand *cand, const u64c *cnt, uint64_t cap, int prec, int tile,
                       double *cand_d2, ResDev *res, hipStream_t st);
void launch_pick_cpp(const Prob *probs, const Cand *cand, const u64c *cnt, uint64_t cap, const double *cand_d2,
                     ResDev *res, hipStream_t st);
// out_cnt counts every verified pair within the radius; the first out_cap are
// written to keys/vals (out_cap = 0: count only).
void launch_verify_frnn(const Prob *probs, const Cand *cand, const u64c *cnt, uint64_t cap, int prec, int tile,
                        uint64_t *keys, double *vals, u64c *out_cnt, uint64_t out_cap, ResDev *res,
                        hipStream_t st);
// The same verification for windows of series (closest pair: frnn = false,
// cand_d2 and res as launch_verify_cpp, followed by launch_pick_cpp; radius:
// frnn = true, keys/vals/out_cnt/out_cap as launch_verify_frnn): 16
// candidates per work-group, their terms formed by 16 threads each.
void launch_verify_windows(bool frnn, const Prob *probs, const Cand *cand, const u64c *cnt, uint64_t cap, int prec,
                           int tile, double *cand_d2, uint64_t *keys, double *vals, u64c *out_cnt, uint64_t out_cap,
                           ResDev *res, hipStream_t st);
// Test of the screen bound on the hardware: for every element (row il,
// column jl) of the m tiles of `tiles` dumped by the M_DUMP screen (rows and
// columns past the problem's rows skipped), the canonical d2 (verifier
// arithmetic) into d2_out, the tile's bound into E_out[t], and the largest
// |screen - d2| / E into *ratio_bits (float bits, rounded up; for int8, 0 if
// equal, else infinity).
void launch_sample_check(const Prob *probs, const uint64_t *tiles, int64_t m, int tile, const void *dump, int prec,
                         double *d2_out, double *E_out, unsigned int *ratio_bits, hipStream_t st);
// Sort m (key, value) pairs by key; arrays hold mpad >= m entries (mpad a power
// of two), the tail is overwritten with sentinels.
void launch_sort_pairs(uint64_t *keys, double *vals, int64_t m, int64_t mpad, hipStream_t st);
// The same order by one radix sort, out of place (temp == nullptr: only sets
// *temp_bytes).
hipError_t sort_pairs_radix(void *temp, size_t *temp_bytes, const uint64_t *keys_in, uint64_t *keys_out,
                            const double *vals_in, double *vals_out, int64_t m, hipStream_t st);
// reference-point pruning (mpr.hip)
void launch_ref_dist(const void *X, int dtype, int64_t n, int64_t d, int64_t ld, const int32_t *refs, int q,
                     double f, double *D, hipStream_t st);
hipError_t sort_ref_order(void *temp, size_t *temp_bytes, const double *D0, double *keys_out, int32_t *idx,
                          int32_t *perm, int64_t n, hipStream_t st);
// rz: q * ell doubles of scratch (the projected, z-normalised references).
void launch_ref_dist_windows(const float *T, int64_t N, int64_t ell, const int32_t *refs, int q, double f,
                             double *rz, double *D, hipStream_t st);
// Encoders of the string problems (encode.hip). Z: rows of Lz int8 values,
// zeroed by the caller; flags: F_SYMBOL for a symbol outside the alphabet.
void launch_encode_strings(const signed char *S, int64_t n, int64_t k, int64_t ld, int sigma, int complement,
                           signed char *Z, int64_t Lz, int64_t split, unsigned int *flags, hipStream_t st);
void launch_check_symbols(const signed char *S, int64_t n, int64_t k, int64_t ld, int sigma, unsigned int *flags,
                          hipStream_t st);
void launch_encode_two_locus(const signed char *G, int64_t m1, int64_t m2, int64_t n, int64_t ld, int direction,
                             signed char *Z, int64_t Lz, int64_t split, unsigned int *flags, hipStream_t st);
// Light-bulb bucketing (lightbulb.hip), B iterations at once. Rows: the n
// strings (mode 0) or their one-hot codes and complements (mode 1, 2n rows:
// `total`); iteration b's keys (ncols chosen columns, bits_per bits each) and
// rows fill [b total, (b+1) total) of keys/rows. The sort orders each
// iteration's part: keys tagged with b above their bits, else a segmented
// sort (seg: B + 1 offsets b total). lb_count: pairs per
// sorted position (num), their exclusive prefix sum over the batch (off;
// rocPRIM scan with temp_bytes >= lb_scan_bytes) and the pairs of each
// iteration (segcnt[B]); lb_fill writes the pairs of positions [p0, p1) to
// cand[off[p] - base ...]; lb_verify merges the exact match counts of
// cand[0, m) into the packed best pair (see the kernels).
void launch_lb_keys(const signed char *S, int64_t n, int64_t ld, int sigma, int mode, int bits_per,
                    const int32_t *cols, int ncols, int B, uint64_t *keys, int32_t *rows, hipStream_t st);
hipError_t lb_sort(void *temp, size_t *temp_bytes, const uint64_t *keys_in, uint64_t *keys_out, const int32_t *rows_in,
                   int32_t *rows_out, int64_t total, int B, const int32_t *seg, int key_bits, hipStream_t st);
size_t lb_scan_bytes(int64_t all);
void launch_lb_count(const uint64_t *keys, const int32_t *rows, int64_t total, int B, int64_t n, int mode,
                     uint64_t *num, uint64_t *off, void *temp, size_t temp_bytes, uint64_t *segcnt, hipStream_t st);
void launch_lb_fill(const uint64_t *keys, const int32_t *rows, int64_t total, int64_t p0, int64_t p1, int64_t n,
                    int mode, const uint64_t *off, uint64_t base, int2 *cand, hipStream_t st);
void launch_lb_verify(const signed char *S, int64_t k, int64_t ld, int mode, const int2 *cand, uint64_t m,
                      unsigned long long *best, hipStream_t st);
void launch_perm_finish(int32_t *perm, int32_t *iperm, int64_t n, int64_t npad, hipStream_t st);
hipError_t sort_ref_order2(void *temp, size_t *temp_bytes, const double *D0, const double *D1, double w,
                           double *keys_out, int32_t *idx, int32_t *perm, int64_t n, hipStream_t st);
int64_t prune_segments(int64_t nT, int64_t G);
// neighbour lists from a pair list (csr.hip): device scratch of the returned
// size (8-byte aligned) plus sort_bytes for the library sorts and scans
size_t csr_scratch_bytes(int64_t m, int64_t n, size_t *sort_bytes);
hipError_t launch_pairs_to_csr(const int64_t *pairs, int64_t m, int64_t n, int64_t *row_ptr, int64_t *cols,
                               void *scratch, void *sort_tmp, size_t sort_bytes, unsigned int *bad, hipStream_t st);
// The pruned tile list of one problem on the device (temp == nullptr: only
// sets *temp_bytes). cnt, off: prune_segments(nT, G) words each; out:
// nT (nT + 1) / 2 + 8 entries; out4 (device): entries, full slots, full
// tiles, partial tiles. Threshold T_host, or from u_bits and r2.
hipError_t launch_prune_list(void *temp, size_t *temp_bytes, const double *lo, const double *hi, int q, int64_t n,
                             int64_t excl, int tile, bool permuted, int64_t G, double T_host,
                             const unsigned long long *u_bits, double r2, uint64_t *cnt, uint64_t *off, uint64_t *out,
                             int64_t *out4, hipStream_t st);
void launch_block_range(const double *D, int64_t n, int q, const int32_t *perm, int tile, int64_t nblk, double *lo,
                        double *hi, hipStream_t st);
// Unpack sorted keys (i << 32 | j) into int64 pairs [m][2] and copy values.
void launch_emit_pairs(const uint64_t *keys, const double *vals, int64_t m, int64_t *pairs, double *d2,
                       hipStream_t st);

// Debug: one 32x32 MFMA block through the screen's fragment path.
void launch_mfma_peak(int prec, int iters, int grid, float *out, hipStream_t st);
void launch_mfma_probe(int prec, const void *A, const void *B, float *C, hipStream_t st);

}  // namespace cpmi
