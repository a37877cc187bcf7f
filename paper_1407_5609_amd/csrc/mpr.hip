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
#include <rocprim/device/device_scan.hpp>

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

// Second key of the two-reference order: the bucket floor(D0 / w) of the row
// sorted k-th by D1 (idx1[k]); the row index rides along.
__global__ void bucket_key_kernel(const double *D0, const int32_t *idx1, double w, int64_t n, uint32_t *key,
                                  int32_t *idx)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = idx1[k];
        const double b = floor(D0[r] / w);
        key[k] = b >= 4294967295.0 ? 0xffffffffu : (uint32_t)fmax(b, 0.0);
        idx[k] = r;
    }
}

// ---- the pruned tile list on the device (MPR step 5 applied to tiles)
//
// Tiles (I, J), I <= J, are enumerated in bands of G block rows, column by
// column within a band (rows ascending): the order the screen's list uses. A
// segment is one column J of one band: at most G tiles. Segment s of band bi
// is column b0 + (s - segoff(bi)), b0 = bi G, with
// segoff(bi) = bi nT - G bi (bi - 1) / 2 segments before band bi.
struct SegMap {
    int64_t nT, G, nB;
    __device__ int64_t segoff(int64_t bi) const { return bi * nT - G * bi * (bi - 1) / 2; }
    __device__ void at(int64_t s, int64_t &b0, int64_t &J) const
    {
        int64_t a = 0, b = nB - 1;   // the last band whose offset is <= s
        while (a < b) {
            const int64_t m = (a + b + 1) / 2;
            if (segoff(m) <= s) a = m;
            else b = m - 1;
        }
        b0 = a * G;
        J = b0 + (s - segoff(a));
    }
};

struct PruneTest {
    const double *lo, *hi;
    int q;
    double T;
    int64_t n, excl;
    int tile;
    bool permuted;
    // the widened intervals of blocks I and J come more than T apart for some
    // reference (the host's rule, operation for operation: a widening by
    // 2^-34 |hi| on both sides)
    __device__ bool far(int64_t I, int64_t J) const
    {
        if (T < 0.0) return true;
        for (int k = 0; k < q; ++k) {
            const double hI = hi[I * q + k], hJ = hi[J * q + k];
            const double mI = 0x1p-34 * fabs(hI), mJ = 0x1p-34 * fabs(hJ);
            const double lwI = lo[I * q + k] - mI, hwI = hI + mI;
            const double lwJ = lo[J * q + k] - mJ, hwJ = hJ + mJ;
            if ((lwJ - hwI > T) | (lwI - hwJ > T)) return true;
        }
        return false;
    }
    // 0: no admissible pair or pruned; 1: kept, every pair admissible; 2: kept, partial
    __device__ int kind(int64_t I, int64_t J) const
    {
        const int64_t maxj = min(J * tile + tile - 1, n - 1);
        if (!permuted && maxj - I * tile < excl) return 0;
        if (far(I, J)) return 0;
        const bool full = !permuted && (J * tile - (I * tile + tile - 1) >= excl) && ((I + 1) * tile <= n) &&
                          ((J + 1) * tile <= n);
        return full ? 1 : 2;
    }
};

// The threshold: T_host, or sqrt(max(r2, U)) (1 + 2^-30) with U the least
// squared distance a previous search left in *u_bits (double bits; not a
// finite number: none found, keep every tile).
__device__ double prune_threshold(double T_host, const unsigned long long *u_bits, double r2)
{
    if (!u_bits) return T_host;
    double u = __longlong_as_double((long long)*u_bits);
    if (!isfinite(u)) u = INFINITY;
    return sqrt(fmax(r2, u)) * (1.0 + 0x1p-30);
}

// Per segment: kept full tiles << 32 | kept partial tiles.
__global__ __launch_bounds__(256) void prune_count_kernel(SegMap sm, PruneTest pt, double T_host,
                                                          const unsigned long long *u_bits, double r2, int64_t S,
                                                          uint64_t *cnt)
{
    pt.T = prune_threshold(T_host, u_bits, r2);
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x) {
        int64_t b0, J;
        sm.at(s, b0, J);
        uint64_t cf = 0, cp = 0;
        for (int64_t I = b0; I < min(b0 + sm.G, sm.nT) && I <= J; ++I) {
            const int k = pt.kind(I, J);
            cf += k == 1;
            cp += k == 2;
        }
        cnt[s] = cf << 32 | cp;
    }
}

// Writes the list: the Tf kept full tiles split into 8 contiguous chunks of
// C = ceil(Tf / 8) interleaved slot by slot (the chunk of slot x is x % 8, so
// the work-groups of one XCD walk one chunk), the empty slots of that part
// TILE_NONE, then the Tp partial tiles in order. out4 = {entries, full
// slots (8 C), Tf, Tp}.
__global__ __launch_bounds__(256) void prune_write_kernel(SegMap sm, PruneTest pt, double T_host,
                                                          const unsigned long long *u_bits, double r2, int64_t S,
                                                          const uint64_t *cnt, const uint64_t *off, uint64_t *out,
                                                          int64_t *out4)
{
    pt.T = prune_threshold(T_host, u_bits, r2);
    const uint64_t tot = off[S - 1] + cnt[S - 1];
    const int64_t Tf = (int64_t)(tot >> 32), Tp = (int64_t)(tot & 0xffffffffu);
    const int64_t C = (Tf + 7) / 8;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < S; s += (int64_t)gridDim.x * blockDim.x) {
        if (s == 0) {
            for (int64_t ch = 0; ch < 8; ++ch)
                for (int64_t pos = max<int64_t>(0, Tf - ch * C); pos < C; ++pos) out[pos * 8 + ch] = TILE_NONE;
            out4[0] = 8 * C + Tp;
            out4[1] = 8 * C;
            out4[2] = Tf;
            out4[3] = Tp;
        }
        int64_t b0, J;
        sm.at(s, b0, J);
        int64_t rf = (int64_t)(off[s] >> 32), rp = (int64_t)(off[s] & 0xffffffffu);
        for (int64_t I = b0; I < min(b0 + sm.G, sm.nT) && I <= J; ++I) {
            const int k = pt.kind(I, J);
            if (k == 0) continue;
            const uint64_t e = tile_pack(0u, (uint32_t)I, (uint32_t)J);
            if (k == 1) {
                out[(rf % C) * 8 + rf / C] = e;
                ++rf;
            } else {
                out[8 * C + rp] = e;
                ++rp;
            }
        }
    }
}

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

// The two-reference order: rows sorted by bucket floor(D0 / w), and by D1
// within a bucket (two stable radix sorts: by D1, then by the bucket).
// keys_out (n doubles) and idx (n int64 = 2n int32) are scratch.
hipError_t sort_ref_order2(void *temp, size_t *temp_bytes, const double *D0, const double *D1, double w,
                           double *keys_out, int32_t *idx, int32_t *perm, int64_t n, hipStream_t st)
{
    int32_t *idx1 = idx + n;                       // rows by D1
    uint32_t *bkey = (uint32_t *)keys_out, *bkey_out = bkey + n;
    if (!temp) {
        size_t a = 0, b = 0;
        hipError_t e = rocprim::radix_sort_pairs(nullptr, a, D1, keys_out, (const int32_t *)idx, idx1,
                                                 (unsigned int)n, 0, 64, st);
        if (e != hipSuccess) return e;
        e = rocprim::radix_sort_pairs(nullptr, b, (const uint32_t *)bkey, bkey_out, (const int32_t *)idx, perm,
                                      (unsigned int)n, 0, 32, st);
        *temp_bytes = std::max(a, b);
        return e;
    }
    hipLaunchKernelGGL(iota_kernel, dim3(grid_of(n, 256)), dim3(256), 0, st, idx, n);
    hipError_t e = rocprim::radix_sort_pairs(temp, *temp_bytes, D1, keys_out, (const int32_t *)idx, idx1,
                                             (unsigned int)n, 0, 64, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bucket_key_kernel, dim3(grid_of(n, 256)), dim3(256), 0, st, D0, (const int32_t *)idx1, w, n,
                       bkey, idx);
    return rocprim::radix_sort_pairs(temp, *temp_bytes, (const uint32_t *)bkey, bkey_out, (const int32_t *)idx, perm,
                                     (unsigned int)n, 0, 32, st);
}

// Segments of the pruned list's enumeration (nT block rows, bands of G).
int64_t prune_segments(int64_t nT, int64_t G)
{
    const int64_t nB = (nT + G - 1) / G;
    return nB * nT - G * nB * (nB - 1) / 2;
}

hipError_t launch_prune_list(void *temp, size_t *temp_bytes, const double *lo, const double *hi, int q, int64_t n,
                             int64_t excl, int tile, bool permuted, int64_t G, double T_host,
                             const unsigned long long *u_bits, double r2, uint64_t *cnt, uint64_t *off, uint64_t *out,
                             int64_t *out4, hipStream_t st)
{
    const int64_t nT = (n + tile - 1) / tile;
    const int64_t S = prune_segments(nT, G);
    if (!temp)
        return rocprim::exclusive_scan(nullptr, *temp_bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                       (uint64_t)0, (size_t)S, rocprim::plus<uint64_t>(), st);
    SegMap sm{nT, G, (nT + G - 1) / G};
    PruneTest pt{lo, hi, q, 0.0, n, excl, tile, permuted};
    const dim3 g(grid_of(S, 256)), b(256);
    hipLaunchKernelGGL(prune_count_kernel, g, b, 0, st, sm, pt, T_host, u_bits, r2, S, cnt);
    hipError_t e = rocprim::exclusive_scan(temp, *temp_bytes, (const uint64_t *)cnt, off, (uint64_t)0, (size_t)S,
                                           rocprim::plus<uint64_t>(), st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(prune_write_kernel, g, b, 0, st, sm, pt, T_host, u_bits, r2, S, (const uint64_t *)cnt,
                       (const uint64_t *)off, out, out4);
    return hipGetLastError();
}

void launch_block_range(const double *D, int64_t n, int q, const int32_t *perm, int tile, int64_t nblk, double *lo,
                        double *hi, hipStream_t st)
{
    hipLaunchKernelGGL(block_range_kernel, dim3((unsigned)nblk), dim3(256), 0, st, D, n, q, perm, tile, lo, hi);
}

}  // namespace cpmi
