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
// One wave per point; lanes across coordinates.
template <typename T>
__global__ __launch_bounds__(256) void ref_dist_kernel(const T *X, int64_t n, int64_t d, int64_t ld,
                                                       const int32_t *refs, int q, double f, double *D)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const T *x = X + i * ld;
    for (int k = 0; k < q; ++k) {
        const T *r = X + (int64_t)refs[k] * ld;
        double s = 0.0;
        for (int64_t c = lane; c < d; c += 64) {
            const double t = f * val(r, c) - val(x, c);
            s = fma(t, t, s);
        }
        s = wave_sum_d(s);
        if (lane == 0) D[(int64_t)k * n + i] = sqrt(s);
    }
}

// Sort keys for the order by distance to reference 0: the bits of a
// non-negative double order like the double; the value carries the index.
__global__ void ref_keys_kernel(const double *D0, int64_t n, uint64_t *keys, double *vals)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        keys[i] = (uint64_t)__double_as_longlong(D0[i]);
        vals[i] = (double)i;
    }
}

__global__ void perm_from_sorted_kernel(const double *vals, int64_t n, int32_t *perm)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        perm[r] = (int32_t)vals[r];
}

// Per block of `tile` screen rows and reference k: the interval of distances,
// lo[b * q + k], hi[b * q + k]. One thread per (block, reference).
__global__ void block_range_kernel(const double *D, int64_t n, int q, const int32_t *perm, int tile, int64_t nblk,
                                   double *lo, double *hi)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= nblk * q) return;
    const int64_t b = t / q;
    const int k = (int)(t % q);
    double mn = INFINITY, mx = -INFINITY;
    const int64_t r1 = min(n, (b + 1) * tile);
    for (int64_t r = b * tile; r < r1; ++r) {
        const double v = D[(int64_t)k * n + perm[r]];
        mn = fmin(mn, v);
        mx = fmax(mx, v);
    }
    lo[t] = mn;
    hi[t] = mx;
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

void launch_ref_keys(const double *D0, int64_t n, uint64_t *keys, double *vals, hipStream_t st)
{
    hipLaunchKernelGGL(ref_keys_kernel, dim3(grid_of(n, 256)), dim3(256), 0, st, D0, n, keys, vals);
}

void launch_perm_from_sorted(const double *vals, int64_t n, int32_t *perm, hipStream_t st)
{
    hipLaunchKernelGGL(perm_from_sorted_kernel, dim3(grid_of(n, 256)), dim3(256), 0, st, vals, n, perm);
}

void launch_block_range(const double *D, int64_t n, int q, const int32_t *perm, int tile, int64_t nblk, double *lo,
                        double *hi, hipStream_t st)
{
    const int64_t t = nblk * q;
    hipLaunchKernelGGL(block_range_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, st, D, n, q, perm, tile,
                       nblk, lo, hi);
}

}  // namespace cpmi
