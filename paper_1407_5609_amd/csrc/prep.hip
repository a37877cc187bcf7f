// Builders of the screen operands.
//
// Points (row preparation): each float32 row x is copied into the screen
// operand x~ (FP32 as is, BF16 rounded to nearest even) or kept as int8, and
// the row scalars used by the epilogue and by the error bound are formed:
// s^ = fp32(||x||^2) and upper bounds of ||x||, ||x~||, ||x - x~||. Block
// maxima of those four values are accumulated per `tile` rows.
//
// Series (l-mer builder): the l-mers T_i = a_i .. a_{i+l-1} (Section 2) are
// z-normalised with the canonical two-pass FP64 arithmetic (ascending sums,
// population variance, correctly rounded division and square root), so the
// verifier can later rebuild the exact canonical window from (T, mu, sigma).
// The normalised window is then rounded into the screen operand as above.
//
// Compiled with -ffp-contract=off: every a*b+c below is either an explicit fma
// or two separately rounded operations, as the canonical definition requires.
#include "bound.h"
#include "cpmi_internal.h"
#include "layout256.h"

namespace cpmi {

__device__ __forceinline__ unsigned short f32_to_bf16_rne(float x)
{
    // branch-free: round to nearest even, except NaN (kept a NaN, quiet if
    // its payload lies in the dropped bits); infinities round to themselves
    const unsigned int u = __float_as_uint(x);
    const unsigned int r = (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
    const unsigned int nan = (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
    return (unsigned short)(((u & 0x7fffffffu) > 0x7f800000u) ? nan : r);
}

__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

// One DPP step on a double: t = v of the lane that `ctrl` selects (0.0 in a
// lane outside row_mask), returned as v + t.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_add(double v)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)u, CTRL, ROW_MASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(u >> 32), CTRL, ROW_MASK, 0xf, false);
    return v + __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over the wave, returned in every lane (any summation order: the row
// terms that use it are bounds). Within each row of 16 lanes: quad_perm
// [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror, after which
// every lane holds its row's sum; then row_bcast:15 into rows 1 and 3 and
// row_bcast:31 into rows 2 and 3 leave the total in lane 63.
__device__ __forceinline__ double wave_sum(double v)
{
    v = dpp_add<0xb1, 0xf>(v);
    v = dpp_add<0x4e, 0xf>(v);
    v = dpp_add<0x141, 0xf>(v);
    v = dpp_add<0x140, 0xf>(v);
    v = dpp_add<0x142, 0xa>(v);
    v = dpp_add<0x143, 0xc>(v);
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 63);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Upper bound as float of a non-negative double (covers the double's own
// rounding with a relative 2^-40 margin).
__device__ __forceinline__ float up_f32(double x) { return f32_up(x * (1.0 + 0x1p-40)); }

__device__ __forceinline__ void atomic_max_f32(float *p, float v)
{
    // non-negative floats order like their bit patterns
    atomicMax((unsigned int *)p, __float_as_uint(v));
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void fill_u64_kernel(uint64_t *p, uint64_t v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void reset_res_kernel(ResDev *r, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        ResDev z;
        z.best_d2 = ~0ull;
        z.best_ij = ~0ull;
        z.err_bits = 0;
        z.ratio_bits = 0;
        z.bound_bits = 0;
        z.flags = 0;
        r[i] = z;
    }
}

// Plain copy of n16 16-byte words; a reference of known traffic for the
// hardware byte counters (each word is read once and written once).
typedef unsigned int cu32x4 __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void calib_copy_kernel(const cu32x4 *__restrict__ src, cu32x4 *__restrict__ dst,
                                                         int64_t n16)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n16; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

static unsigned grid_for(int64_t n, int per)
{
    int64_t g = (n + per - 1) / per;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, v, n);
}
void launch_fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, p, v, n);
}
void launch_calib_copy(const void *src, void *dst, int64_t n16, hipStream_t st)
{
    if (n16 > 0)
        hipLaunchKernelGGL(calib_copy_kernel, dim3(grid_for(n16, 256 * 8)), dim3(256), 0, st, (const cu32x4 *)src,
                           (cu32x4 *)dst, n16);
}
void launch_reset_res(ResDev *r, int64_t n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(reset_res_kernel, dim3(grid_for(n, 256)), dim3(256), 0, st, r, n);
}

// Element index of element k of row r in the screen operand (rows of kpad
// elements of esz bytes): row-major for the 128-row screen, slice-major per
// 256-row block for the 256-row screen (layout256.h).
__device__ __forceinline__ int64_t xs_index(int64_t r, int64_t k, int32_t kpad, int esz, int tile)
{
    if (tile != 256) return r * (int64_t)kpad + k;
    return l256::xs_offset(r, k * esz, (int64_t)kpad * esz) / esz;
}

// ---------------------------------------------------------------------------
// points: a work-group of 256 threads prepares PREP_ROWS consecutive rows, one
// wave per row at a time; the block maxima of its rows are reduced in LDS and
// merged with one set of atomics per work-group (the rows of a work-group lie
// in one tile block), not one per row: per-row atomics on the few addresses
// of the blocks in flight serialise.
// ---------------------------------------------------------------------------
constexpr int PREP_ROWS = 32;   // divides every tile edge and every npad

template <int PREC, bool INT8_IN>
__global__ __launch_bounds__(256) void prep_points_kernel(const void *pts, int64_t n, int64_t d, int64_t ld,
                                                          void *xs, int32_t kpad, int64_t npad, void *shat,
                                                          float4 *bmax, int tile, unsigned int *flags,
                                                          const int32_t *perm, uint2 *fold, float4 *rowstat)
{
    __shared__ float4 sh_bm[4];
    __shared__ unsigned int sh_f[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * PREP_ROWS;
    // four consecutive coordinates per lane, 256 per step (kpad is a multiple
    // of 32; four elements never straddle a 64-byte slice of the operand);
    // vector loads when the rows are 16-byte aligned
    const bool vec = ((ld & 3) == 0) && (((uintptr_t)pts & 15) == 0);
    float4 bm = make_float4(0.f, 0.f, 0.f, 0.f);
    unsigned int fl = 0;
    for (int q = wave; q < PREP_ROWS; q += 4) {
        const int64_t row = r0 + q;
        const bool real = row < n;
        // screen row `row` holds source row srow (a permutation of 0..n-1, or the identity)
        const int64_t srow = (real && perm) ? (int64_t)perm[row] : row;
        if constexpr (INT8_IN) {
            const signed char *x = (const signed char *)pts + srow * ld;
            const bool vec8 = ((ld & 3) == 0) && (((uintptr_t)pts & 3) == 0);
            int s = 0;
#pragma unroll 2
            for (int64_t k0 = 4 * lane; k0 < kpad; k0 += 256) {
                signed char v[4];
                if (real && vec8 && k0 + 4 <= d) {
                    const int qv = *(const int *)(x + k0);
#pragma unroll
                    for (int u = 0; u < 4; ++u) v[u] = (signed char)(qv >> (8 * u));
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u) v[u] = (real && k0 + u < d) ? x[k0 + u] : (signed char)0;
                }
                int packed = 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    packed |= (int)(unsigned char)v[u] << (8 * u);
                    s += (int)v[u] * (int)v[u];
                }
                *(int *)((signed char *)xs + xs_index(row, k0, kpad, 1, tile)) = packed;
            }
#pragma unroll
            for (int of = 32; of > 0; of >>= 1) s += __shfl_xor(s, of, 64);
            if (lane == 0) ((int *)shat)[row] = s;
        } else {
            const float *x = (const float *)pts + srow * ld;
            double s = 0.0, t2 = 0.0, r2 = 0.0;
            bool bad = false;
#pragma unroll 2
            for (int64_t k0 = 4 * lane; k0 < kpad; k0 += 256) {
                float v[4];
                if (real && vec && k0 + 4 <= d) {
                    const float4 qv = *(const float4 *)(x + k0);
                    v[0] = qv.x;
                    v[1] = qv.y;
                    v[2] = qv.z;
                    v[3] = qv.w;
                } else {
#pragma unroll
                    for (int u = 0; u < 4; ++u) v[u] = (real && k0 + u < d) ? x[k0 + u] : 0.0f;
                }
                float vt[4];
                if constexpr (PREC == P_BF16) {
                    unsigned short h[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        h[u] = f32_to_bf16_rne(v[u]);
                        vt[u] = bf16_to_f32(h[u]);
                    }
                    const uint2 pk = make_uint2((uint32_t)h[0] | ((uint32_t)h[1] << 16),
                                                (uint32_t)h[2] | ((uint32_t)h[3] << 16));
                    *(uint2 *)((unsigned short *)xs + xs_index(row, k0, kpad, 2, tile)) = pk;
                } else {
                    *(float4 *)((float *)xs + xs_index(row, k0, kpad, 4, tile)) =
                        make_float4(v[0], v[1], v[2], v[3]);
#pragma unroll
                    for (int u = 0; u < 4; ++u) vt[u] = v[u];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    bad |= !isfinite(v[u]);
                    const double vd = (double)v[u], vtd = (double)vt[u];
                    s = fma(vd, vd, s);
                    t2 = fma(vtd, vtd, t2);
                    const double df = vd - vtd;  // exact: both are float values
                    r2 = fma(df, df, r2);
                }
            }
            s = wave_sum(s);
            t2 = wave_sum(t2);
            r2 = wave_sum(r2);
            const unsigned long long anybad = __ballot(bad);
            if (lane == 0) {
                ((float *)shat)[row] = (float)s;
                if (fold) fold[row] = fold_words((float)s);
                const float4 v = make_float4(f32_up(s), up_f32(sqrt(s)), up_f32(sqrt(t2)), up_f32(sqrt(r2)));
                if (rowstat) rowstat[row] = v;
                bm.x = fmaxf(bm.x, v.x);
                bm.y = fmaxf(bm.y, v.y);
                bm.z = fmaxf(bm.z, v.z);
                bm.w = fmaxf(bm.w, v.w);
                if (anybad) fl |= F_NONFINITE;
                if (!(s < 0x1p100)) fl |= F_RANGE;
            }
        }
    }
    if constexpr (!INT8_IN) {
        if (lane == 0) {
            sh_bm[wave] = bm;
            sh_f[wave] = fl;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            float4 m = sh_bm[0];
            unsigned int f = sh_f[0];
            for (int w = 1; w < 4; ++w) {
                m.x = fmaxf(m.x, sh_bm[w].x);
                m.y = fmaxf(m.y, sh_bm[w].y);
                m.z = fmaxf(m.z, sh_bm[w].z);
                m.w = fmaxf(m.w, sh_bm[w].w);
                f |= sh_f[w];
            }
            float *b = (float *)(bmax + r0 / tile);
            atomic_max_f32(b + 0, m.x);
            atomic_max_f32(b + 1, m.y);
            atomic_max_f32(b + 2, m.z);
            atomic_max_f32(b + 3, m.w);
            if (f) atomicOr(flags, f);
        }
    }
}

void launch_prep_points(const void *pts, int dtype, int64_t n, int64_t d, int64_t ld, int prec, void *xs,
                        int32_t kpad, int64_t npad, void *shat, float4 *bmax, int tile, unsigned int *flags,
                        const int32_t *perm, uint2 *fold, float4 *rowstat, hipStream_t st)
{
    dim3 g((unsigned)(npad / PREP_ROWS)), b(256);
    if (dtype == 1)
        hipLaunchKernelGGL((prep_points_kernel<P_I8, true>), g, b, 0, st, pts, n, d, ld, xs, kpad, npad, shat, bmax,
                           tile, flags, perm, nullptr, nullptr);
    else if (prec == P_BF16)
        hipLaunchKernelGGL((prep_points_kernel<P_BF16, false>), g, b, 0, st, pts, n, d, ld, xs, kpad, npad, shat,
                           bmax, tile, flags, perm, fold, rowstat);
    else
        hipLaunchKernelGGL((prep_points_kernel<P_F32, false>), g, b, 0, st, pts, n, d, ld, xs, kpad, npad, shat,
                           bmax, tile, flags, perm, nullptr, rowstat);
}

// ---------------------------------------------------------------------------
// series, in two kernels. Statistics: a block of 256 threads takes 256
// consecutive windows of one job (four builder blocks; a job holds a whole
// number of them), a thread per window, with the stretch of the series they
// cover (256 + ell - 1 values, ell <= 8192) staged in LDS: canonical mean and
// sigma, each a sequential sum in k. Every window's chain of dependent
// additions runs at once, in all four waves. Operand: a block of 256 threads
// builds SERIES_WPB (64) consecutive windows, a lane per window and a quarter
// of the elements per wave, in 16-byte chunks: normalised values, screen
// operand and row scalars (the quarters' sums meet in LDS, no wave
// reductions).
// ---------------------------------------------------------------------------
constexpr int STATS_W = 4 * SERIES_WPB;

// Job of builder block bid: the last job with blk_base <= bid.
__device__ __forceinline__ int64_t job_of(const SeriesJob *jobs, int64_t njobs, int64_t bid)
{
    int64_t lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (jobs[mid].blk_base <= bid) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ __launch_bounds__(256) void series_stats_kernel(const SeriesJob *jobs, int64_t njobs)
{
    __shared__ float sh_T[STATS_W + SERIES_MAX_ELL];
    const int64_t bid = (int64_t)blockIdx.x * (STATS_W / SERIES_WPB);
    const SeriesJob J = jobs[job_of(jobs, njobs, bid)];
    const int64_t N = J.len - J.ell + 1;
    const int64_t w0 = (bid - J.blk_base) * SERIES_WPB;
    const int tid = threadIdx.x;
    const int64_t ell = J.ell;
    const int64_t span = w0 < N ? min<int64_t>(STATS_W + ell - 1, J.len - w0) : 0;
    for (int64_t k = tid; k < span; k += 256) sh_T[k] = J.T[w0 + k];
    __syncthreads();
    const int64_t w = w0 + tid;
    if (w >= N) return;
    // sequential in k; the LDS reads of eight terms are issued before their
    // additions
    const float *tw = sh_T + tid;   // T[w + k] = tw[k]
    double s = 0.0;
    bool bad = false;
    int64_t k = 0;
    for (; k + 8 <= ell; k += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = tw[k + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            bad |= !isfinite(v[u]);
            s += (double)v[u];
        }
    }
    for (; k < ell; ++k) {
        bad |= !isfinite(tw[k]);
        s += (double)tw[k];
    }
    const double mu = s / (double)ell;
    double v2 = 0.0;
    for (k = 0; k + 8 <= ell; k += 8) {
        float v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = tw[k + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double e = (double)v[u] - mu;
            v2 = fma(e, e, v2);
        }
    }
    for (; k < ell; ++k) {
        const double e = (double)tw[k] - mu;
        v2 = fma(e, e, v2);
    }
    const double sg = sqrt(v2 / (double)ell);
    J.mu[w] = mu;
    J.sigma[w] = sg;
    unsigned int f = 0;
    if (bad) f |= F_NONFINITE;
    if (!(sg > 0.0)) f |= F_DEGENERATE;
    if (f) atomicOr(J.flags, f);
}

template <int PREC>
__global__ __launch_bounds__(256) void prep_series_kernel(const SeriesJob *jobs, int64_t njobs, int tile)
{
    constexpr int ESZ = PREC == P_BF16 ? 2 : 4;
    constexpr int CH = 16 / ESZ;   // elements per 16-byte store
    __shared__ double sh_mu[SERIES_WPB];
    __shared__ double sh_inv[SERIES_WPB];
    __shared__ float sh_T[SERIES_WPB + SERIES_MAX_ELL];
    __shared__ double sh_part[3][4][SERIES_WPB];
    const int64_t bid = blockIdx.x;
    const SeriesJob J = jobs[job_of(jobs, njobs, bid)];
    const int64_t N = J.len - J.ell + 1;          // windows
    const int64_t w0 = (bid - J.blk_base) * SERIES_WPB;  // first window of the block
    const int tid = threadIdx.x;
    const int64_t ell = J.ell;
    // values T[w0 .. w0 + span) : every window of the block that exists; zeros
    // after them up to the last element a lane reads (SERIES_WPB + kpad - 1 <=
    // SERIES_WPB + SERIES_MAX_ELL), so that no value read below is left unset
    const int64_t span = w0 < N ? min<int64_t>(SERIES_WPB + ell - 1, J.len - w0) : 0;
    for (int64_t k = tid; k < SERIES_WPB + J.kpad - 1; k += 256) sh_T[k] = k < span ? J.T[w0 + k] : 0.0f;
    if (tid < SERIES_WPB) {
        const int64_t w = w0 + tid;
        const double sg = w < N ? J.sigma[w] : 0.0;
        sh_mu[tid] = w < N ? J.mu[w] : 0.0;
        // one correctly rounded reciprocal per window: the operand's FP64
        // values (T - mu) * inv are within 2^-51 (relative) of the canonical
        // quotients (T - mu) / sigma, which the row terms below absorb; a
        // window that is not real has inv = 0, hence an operand row of zeros
        sh_inv[tid] = sg > 0.0 ? 1.0 / sg : 0.0;
    }
    __syncthreads();

    // lane l: window w0 + l (every block lies inside its job's npad rows);
    // wave v: the quarter [v kpad/4, (v+1) kpad/4) of its elements (a whole
    // number of 16-byte chunks, which never straddle a 64-byte slice)
    const int lane = tid & 63, wave = tid >> 6;
    const int64_t w = w0 + lane;
    const int64_t row = (J.iperm && w < N) ? (int64_t)J.iperm[w] : w;
    const double mu = sh_mu[lane], inv = sh_inv[lane];
    const int ell32 = (int)ell;   // <= SERIES_MAX_ELL: 32-bit element indices
    const int kq = J.kpad / 4;
    const float *tw = sh_T + lane;   // T[w + k] = tw[k]
    double s = 0.0, t2 = 0.0, r2 = 0.0;
    for (int k0 = wave * kq; k0 < (wave + 1) * kq; k0 += CH) {
        double xh[CH];
        float vt[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            // read for every k (past the window the value is dropped)
            const double v = ((double)tw[k0 + u] - mu) * inv;
            xh[u] = (k0 + u < ell32) ? v : 0.0;
        }
        if constexpr (PREC == P_BF16) {
            uint32_t h[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                h[u] = f32_to_bf16_rne((float)xh[u]);
                vt[u] = bf16_to_f32((unsigned short)h[u]);
            }
            *(uint4 *)((unsigned short *)J.xs + xs_index(row, k0, J.kpad, 2, tile)) =
                make_uint4(h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16));
        } else {
#pragma unroll
            for (int u = 0; u < CH; ++u) vt[u] = (float)xh[u];
            *(float4 *)((float *)J.xs + xs_index(row, k0, J.kpad, 4, tile)) = make_float4(vt[0], vt[1], vt[2], vt[3]);
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const double vtd = (double)vt[u];
            s = fma(xh[u], xh[u], s);
            t2 = fma(vtd, vtd, t2);
            const double df = xh[u] - vtd;
            r2 = fma(df, df, r2);
        }
    }
    sh_part[0][wave][lane] = s;
    sh_part[1][wave][lane] = t2;
    sh_part[2][wave][lane] = r2;
    __syncthreads();
    if (wave != 0) return;
    s = (sh_part[0][0][lane] + sh_part[0][1][lane]) + (sh_part[0][2][lane] + sh_part[0][3][lane]);
    t2 = (sh_part[1][0][lane] + sh_part[1][1][lane]) + (sh_part[1][2][lane] + sh_part[1][3][lane]);
    r2 = (sh_part[2][0][lane] + sh_part[2][1][lane]) + (sh_part[2][2][lane] + sh_part[2][3][lane]);
    ((float *)J.shat)[row] = (float)s;
    if (J.fold) J.fold[row] = fold_words((float)s);
    // r: distance of the operand from the canonical window, widened by
    // 2^-50 ||x|| for the reciprocal's rounding (the norms carry the 2^-40
    // widening of up_f32, which covers it)
    float4 v = make_float4(f32_up(s), up_f32(sqrt(s)), up_f32(sqrt(t2)), up_f32(sqrt(r2) + 0x1p-50 * sqrt(s)));
    if (J.rowstat) J.rowstat[row] = v;
    // windows in reference order land in any tile block: their per-row terms
    // are reduced per block afterwards (launch_block_max)
    if (J.iperm) return;
    // windows in position order: the block's SERIES_WPB rows lie in one tile
    // block; one set of atomics per work-group (per-window atomics on the few
    // block addresses in flight serialise)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v.x = fmaxf(v.x, __shfl_xor(v.x, o, 64));
        v.y = fmaxf(v.y, __shfl_xor(v.y, o, 64));
        v.z = fmaxf(v.z, __shfl_xor(v.z, o, 64));
        v.w = fmaxf(v.w, __shfl_xor(v.w, o, 64));
    }
    if (lane == 0) {
        float *bm = (float *)(J.bmax + w0 / tile);
        atomic_max_f32(bm + 0, v.x);
        atomic_max_f32(bm + 1, v.y);
        atomic_max_f32(bm + 2, v.z);
        atomic_max_f32(bm + 3, v.w);
    }
}

__global__ __launch_bounds__(256) void block_max_kernel(const float4 *rowstat, int tile, float4 *bmax)
{
    __shared__ float4 red[4];
    const int64_t b = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    float4 v = t < tile ? rowstat[b * tile + t] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        v.x = fmaxf(v.x, __shfl_xor(v.x, o, 64));
        v.y = fmaxf(v.y, __shfl_xor(v.y, o, 64));
        v.z = fmaxf(v.z, __shfl_xor(v.z, o, 64));
        v.w = fmaxf(v.w, __shfl_xor(v.w, o, 64));
    }
    if (lane == 0) red[wave] = v;
    __syncthreads();
    if (t == 0) {
        float4 m = red[0];
        for (int w = 1; w < 4; ++w) {
            m.x = fmaxf(m.x, red[w].x);
            m.y = fmaxf(m.y, red[w].y);
            m.z = fmaxf(m.z, red[w].z);
            m.w = fmaxf(m.w, red[w].w);
        }
        bmax[b] = m;
    }
}

void launch_block_max(const float4 *rowstat, int64_t npad, int tile, float4 *bmax, hipStream_t st)
{
    hipLaunchKernelGGL(block_max_kernel, dim3((unsigned)(npad / tile)), dim3(256), 0, st, rowstat, tile, bmax);
}

void launch_prep_series(const SeriesJob *jobs, int64_t njobs, int64_t total_blocks, int prec, int tile,
                        hipStream_t st)
{
    if (total_blocks <= 0) return;
    // jobs hold whole 256-window blocks; a statistics block past the last
    // window has nothing to do
    const int64_t sb = (total_blocks + STATS_W / SERIES_WPB - 1) / (STATS_W / SERIES_WPB);
    hipLaunchKernelGGL(series_stats_kernel, dim3((unsigned)sb), dim3(256), 0, st, jobs, njobs);
    if (prec == P_BF16)
        hipLaunchKernelGGL(prep_series_kernel<P_BF16>, dim3((unsigned)total_blocks), dim3(256), 0, st, jobs, njobs,
                           tile);
    else
        hipLaunchKernelGGL(prep_series_kernel<P_F32>, dim3((unsigned)total_blocks), dim3(256), 0, st, jobs, njobs,
                           tile);
}

}  // namespace cpmi
