// Reference-point tile pruning (the MPR idea of Section 3, applied to tiles).
//
// MPR picks q reference points, projects each one outwards by a factor f
// (every coordinate multiplied by f), computes the distance of every input
// point to every projected reference, and orders the points by their distance
// to the first reference. By the triangle inequality |d(r,x) - d(r,y)| is a
// lower bound of d(x,y) for any reference r. Here the bound is applied to whole
// screen tiles: with the rows in that order, block I's distances to reference
// k lie in [lo_Ik, hi_Ik], so every pair of tile (I, J) is at least
//     LB_IJ = max_k max(0, lo_Jk - hi_Ik, lo_Ik - hi_Jk)
// apart, and a tile whose LB exceeds the closest-pair upper bound (and the
// radius) cannot hold an answer. The kernels below build what the host needs
// to drop such tiles: the distance table, the order and the per-block
// intervals.
//
// Distances here are FP64 sums over lanes (not the canonical order): they
// only feed the pruning test, which allows for their rounding with a margin
// far larger than it (the host side).
#include <algorithm>

#include <rocprim/device/device_radix_sort.hpp>

#include "cpmi_internal.h"

namespace cpmi {

namespace {

__device__ __forceinline__ double wave_sum_d(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T> __device__ __forceinline__ double val(const T *p, int64_t k) { return (double)p[k]; }

// D[k * n + i] = || f * x_ref_k - x_i || for every point i and reference k.
// One wave per point, lanes across coordinates, all references (q <= 32) in
// one sweep over the point.
template <typename T>
__global__ __launch_bounds__(256) void ref_dist_kernel(const T *X, int64_t n, int64_t d, int64_t ld,
                                                       const int32_t *refs, int q, double f, double *D)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const T *x = X + i * ld;
    double s[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) s[k] = 0.0;
    for (int64_t c = lane; c < d; c += 64) {
        const double xv = val(x, c);
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            if (k < q) {
                const double t = f * val(X + (int64_t)refs[k] * ld, c) - xv;
                s[k] = fma(t, t, s[k]);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        if (k < q) {
            const double v = wave_sum_d(s[k]);
            if (lane == 0) D[(int64_t)k * n + i] = sqrt(v);
        }
    }
}

// The q projected references of a series, z-normalised: rz[k * ell + c] =
// f * (T[r_k + c] - mu) / sigma (FP64; mean and sigma by a wave reduction;
// a window of zero variance counts as the zero vector). One wave each.
__global__ __launch_bounds__(64) void ref_windows_kernel(const float *T, int64_t ell, const int32_t *refs, double f,
                                                         double *rz)
{
    const int k = blockIdx.x, lane = threadIdx.x;
    const float *x = T + refs[k];
    double s = 0.0;
    for (int64_t c = lane; c < ell; c += 64) s += (double)x[c];
    const double m = wave_sum_d(s) / (double)ell;
    double v2 = 0.0;
    for (int64_t c = lane; c < ell; c += 64) {
        const double e = (double)x[c] - m;
        v2 = fma(e, e, v2);
    }
    const double sg = sqrt(wave_sum_d(v2) / (double)ell);
    const double sc = sg > 0.0 ? f / sg : 0.0;
    for (int64_t c = lane; c < ell; c += 64) rz[(int64_t)k * ell + c] = ((double)x[c] - m) * sc;
}

// D[k * N + w] = || rz_k - xhat_w || for every window w of the series, xhat_w
// = (T[w + c] - mu_w) / sigma_w, c < ell (a window of zero variance counts as
// the zero vector; the builder reports such a series as an error). A
// work-group takes 64 consecutive windows, a lane each, with the stretch of
// the series they cover staged in LDS; its four waves split the window
// length and their partial sums meet in LDS. The reference values are the
// same across a wave and come in through scalar loads. Mean and sigma here
// are not the builder's canonical ones: the distances only feed the pruning
// test, whose margin covers their rounding.
template <int QM, bool EXACT>
__global__ __launch_bounds__(256) void ref_dist_windows_kernel(const float *T, int64_t N, int64_t ell,
                                                               const double *rz_, int q, double *D)
{
    __shared__ float sh[64 + SERIES_MAX_ELL];
    __shared__ double red[4][64];
    const __attribute__((address_space(4))) double *rz = (const __attribute__((address_space(4))) double *)rz_;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);   // uniform: scalar reference loads
    const int64_t w0 = (int64_t)blockIdx.x * 64;
    const int64_t span = min<int64_t>(64 + ell - 1, N + ell - 1 - w0);   // values of the live windows
    for (int64_t k = threadIdx.x; k < span; k += 256) sh[k] = T[w0 + k];
    __syncthreads();
    const int64_t wl = min<int64_t>(lane, N - 1 - w0);   // this lane's window (the last live one past N)
    const float *x = sh + wl;
    const int64_t part = (ell + 3) / 4;
    const int64_t c0 = min<int64_t>(ell, wave * part), c1 = min<int64_t>(ell, c0 + part);
    // sum of the four waves' partial values v, in every lane of every wave
    auto total = [&](double v) {
        red[wave][lane] = v;
        __syncthreads();
        const double t = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
        __syncthreads();
        return t;
    };
    double s = 0.0;
    for (int64_t c = c0; c < c1; ++c) s += (double)x[c];
    const double m = total(s) / (double)ell;
    double v2 = 0.0;
    for (int64_t c = c0; c < c1; ++c) {
        const double e = (double)x[c] - m;
        v2 = fma(e, e, v2);
    }
    const double sg = sqrt(total(v2) / (double)ell);
    const double inv = sg > 0.0 ? 1.0 / sg : 0.0;
    // reference row of accumulator k: k itself when QM == q, else clamped (the
    // surplus accumulators repeat the last reference and are not stored), so
    // that no branch on q separates the scalar loads of a group of columns
    const __attribute__((address_space(4))) double *rk[QM];
#pragma unroll
    for (int k = 0; k < QM; ++k) rk[k] = rz + (int64_t)(EXACT ? k : min(k, q - 1)) * ell;
    double acc[QM];
#pragma unroll
    for (int k = 0; k < QM; ++k) acc[k] = 0.0;
    int64_t c = c0;
    for (; c + 4 <= c1; c += 4) {
        double xv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) xv[u] = ((double)x[c + u] - m) * inv;
#pragma unroll
        for (int k = 0; k < QM; ++k) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double t = rk[k][c + u] - xv[u];
                acc[k] = fma(t, t, acc[k]);
            }
        }
    }
    for (; c < c1; ++c) {
        const double xv = ((double)x[c] - m) * inv;
#pragma unroll
        for (int k = 0; k < QM; ++k) {
            const double t = rk[k][c] - xv;
            acc[k] = fma(t, t, acc[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < QM; ++k) {
        if (EXACT || k < q) {
            const double v = total(acc[k]);
            if (wave == 0 && w0 + lane < N) D[(int64_t)k * N + w0 + lane] = sqrt(v);
        }
    }
}

// Complete a permutation of 0..n-1 for the screen: its inverse, and the tail
// n..npad-1 (padding rows, which the screen masks by row index) set to 0.
__global__ void perm_finish_kernel(int32_t *perm, int32_t *iperm, int64_t n, int64_t npad)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < npad; r += (int64_t)gridDim.x * blockDim.x) {
        if (r < n) iperm[perm[r]] = (int32_t)r;
        else perm[r] = 0;
    }
}

__global__ void iota_kernel(int32_t *v, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = (int32_t)i;
}

// Per block of `tile` (<= 256) screen rows and reference k: the interval of
// distances, lo[b * q + k], hi[b * q + k]. One work-group of 256 threads per
// block, a thread per row, reduced over the work-group.
__global__ __launch_bounds__(256) void block_range_kernel(const double *D, int64_t n, int q, const int32_t *perm,
                                                          int tile, double *lo, double *hi)
{
    __shared__ double red[2][4];
    const int64_t b = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r = b * tile + tid;
    const bool live = tid < tile && r < n;
    const int64_t src = live ? perm[r] : 0;
    for (int k = 0; k < q; ++k) {
        const double v = live ? D[(int64_t)k * n + src] : 0.0;
        double mn = live ? v : INFINITY, mx = live ? v : -INFINITY;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            mn = fmin(mn, __shfl_xor(mn, o, 64));
            mx = fmax(mx, __shfl_xor(mx, o, 64));
        }
        if (lane == 0) {
            red[0][wave] = mn;
            red[1][wave] = mx;
        }
        __syncthreads();
        if (tid == 0) {
            lo[b * q + k] = fmin(fmin(red[0][0], red[0][1]), fmin(red[0][2], red[0][3]));
            hi[b * q + k] = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
        }
        __syncthreads();
    }
}

unsigned grid_of(int64_t n, int per) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + per - 1) / per, 65536)); }

}  // namespace

void launch_ref_dist(const void *X, int dtype, int64_t n, int64_t d, int64_t ld, const int32_t *refs, int q,
                     double f, double *D, hipStream_t st)
{
    const dim3 g((unsigned)((n + 3) / 4)), b(256);
    if (dtype == 1)
        hipLaunchKernelGGL((ref_dist_kernel<signed char>), g, b, 0, st, (const signed char *)X, n, d, ld, refs, q, f, D);
    else
        hipLaunchKernelGGL((ref_dist_kernel<float>), g, b, 0, st, (const float *)X, n, d, ld, refs, q, f, D);
}

void launch_ref_dist_windows(const float *T, int64_t N, int64_t ell, const int32_t *refs, int q, double f,
                             double *rz, double *D, hipStream_t st)
{
    hipLaunchKernelGGL(ref_windows_kernel, dim3((unsigned)q), dim3(64), 0, st, T, ell, refs, f, rz);
    const dim3 g((unsigned)((N + 63) / 64)), b(256);
    switch (q) {
#define CPMI_RDW(Q) \
    case Q: hipLaunchKernelGGL((ref_dist_windows_kernel<Q, true>), g, b, 0, st, T, N, ell, rz, q, D); break;
        CPMI_RDW(1) CPMI_RDW(2) CPMI_RDW(3) CPMI_RDW(4) CPMI_RDW(5) CPMI_RDW(6) CPMI_RDW(7) CPMI_RDW(8)
        CPMI_RDW(9) CPMI_RDW(10) CPMI_RDW(11) CPMI_RDW(12)
#undef CPMI_RDW
    default:
        if (q <= 16) hipLaunchKernelGGL((ref_dist_windows_kernel<16, false>), g, b, 0, st, T, N, ell, rz, q, D);
        else hipLaunchKernelGGL((ref_dist_windows_kernel<32, false>), g, b, 0, st, T, N, ell, rz, q, D);
    }
}

void launch_perm_finish(int32_t *perm, int32_t *iperm, int64_t n, int64_t npad, hipStream_t st)
{
    hipLaunchKernelGGL(perm_finish_kernel, dim3(grid_of(npad, 256)), dim3(256), 0, st, perm, iperm, n, npad);
}

// The reference order: perm[0..n) = the indices 0..n-1 sorted (stably) by
// D0 (rocPRIM's device radix sort). temp == nullptr only sets *temp_bytes.
// keys_out (n doubles) and idx (n int32) are scratch.
hipError_t sort_ref_order(void *temp, size_t *temp_bytes, const double *D0, double *keys_out, int32_t *idx,
                          int32_t *perm, int64_t n, hipStream_t st)
{
    if (temp) hipLaunchKernelGGL(iota_kernel, dim3(grid_of(n, 256)), dim3(256), 0, st, idx, n);
    return rocprim::radix_sort_pairs(temp, *temp_bytes, D0, keys_out, (const int32_t *)idx, perm, (unsigned int)n, 0,
                                     64, st);
}

void launch_block_range(const double *D, int64_t n, int q, const int32_t *perm, int tile, int64_t nblk, double *lo,
                        double *hi, hipStream_t st)
{
    hipLaunchKernelGGL(block_range_kernel, dim3((unsigned)nblk), dim3(256), 0, st, D, n, q, perm, tile, lo, hi);
}

}  // namespace cpmi
