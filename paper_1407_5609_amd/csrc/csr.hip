// Neighbour lists of a radius search (the output form of MPR-FRNNS, Section
// 3.5: N(i) for every point i, the other points within R) built from the
// canonical pair list (i, j), i < j, on the device.
//
// Each pair is listed under both of its points. With the pairs sorted once by
// (i, j) and once by (j, i), the neighbours of v below v form one run of the
// second order and those above v one run of the first, so row v is that
// first run followed by the second: ascending, with no sort per row and no
// atomics deciding any position.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "cpmi_internal.h"

namespace cpmi {

namespace {

constexpr uint64_t BAD = ~0ull;

unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)); }

// Keys of both orders and the run lengths: cnt_hi[i] counts the pairs whose
// first point is i, cnt_lo[j] those whose second point is j. A pair outside
// 0 <= i < j < n raises *bad and is keyed past every valid one.
__global__ void csr_keys_kernel(const int64_t *pairs, int64_t m, int64_t n, uint64_t *key_hi, uint64_t *key_lo,
                                unsigned long long *cnt_hi, unsigned long long *cnt_lo, unsigned int *bad)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = pairs[2 * k], j = pairs[2 * k + 1];
        if (i < 0 || j >= n || i >= j) {
            atomicOr(bad, 1u);
            key_hi[k] = BAD;
            key_lo[k] = BAD;
            continue;
        }
        key_hi[k] = (uint64_t)i << 32 | (uint64_t)j;
        key_lo[k] = (uint64_t)j << 32 | (uint64_t)i;
        atomicAdd(&cnt_hi[i], 1ull);
        atomicAdd(&cnt_lo[j], 1ull);
    }
}

// row_ptr[v] = (neighbours of all u < v) = off_lo[v] + off_hi[v], v = 0..n
__global__ void csr_rows_kernel(const uint64_t *off_lo, const uint64_t *off_hi, int64_t n, int64_t *row_ptr)
{
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v <= n; v += (int64_t)gridDim.x * blockDim.x)
        row_ptr[v] = (int64_t)(off_lo[v] + off_hi[v]);
}

// Neighbours below v: the run of the (j, i) order with second point v, in
// place at the start of row v.
__global__ void csr_fill_lo_kernel(const uint64_t *sorted_lo, int64_t m, const uint64_t *off_lo,
                                   const int64_t *row_ptr, int64_t *cols)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = sorted_lo[k];
        if (key == BAD) continue;
        const int64_t v = (int64_t)(key >> 32), u = (int64_t)(key & 0xffffffffu);
        cols[row_ptr[v] + (k - (int64_t)off_lo[v])] = u;
    }
}

// Neighbours above v: the run of the (i, j) order with first point v, after
// the neighbours below it.
__global__ void csr_fill_hi_kernel(const uint64_t *sorted_hi, int64_t m, const uint64_t *off_hi,
                                   const unsigned long long *cnt_lo, const int64_t *row_ptr, int64_t *cols)
{
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < m; k += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = sorted_hi[k];
        if (key == BAD) continue;
        const int64_t v = (int64_t)(key >> 32), w = (int64_t)(key & 0xffffffffu);
        cols[row_ptr[v] + (int64_t)cnt_lo[v] + (k - (int64_t)off_hi[v])] = w;
    }
}

}  // namespace

size_t csr_scratch_bytes(int64_t m, int64_t n, size_t *sort_bytes)
{
    size_t a = 0, b = 0;
    rocprim::radix_sort_keys(nullptr, a, (const uint64_t *)nullptr, (uint64_t *)nullptr, (unsigned int)m, 0, 64,
                             (hipStream_t)0);
    rocprim::exclusive_scan(nullptr, b, (const uint64_t *)nullptr, (uint64_t *)nullptr, (uint64_t)0, (size_t)(n + 1),
                            rocprim::plus<uint64_t>(), (hipStream_t)0);
    *sort_bytes = std::max(std::max(a, b), (size_t)1);
    // four key arrays of m, two counts and two offsets of n + 1, the flag
    return ((size_t)4 * m + (size_t)4 * (n + 1)) * 8 + 256;
}

hipError_t launch_pairs_to_csr(const int64_t *pairs, int64_t m, int64_t n, int64_t *row_ptr, int64_t *cols,
                               void *scratch, void *sort_tmp, size_t sort_bytes, unsigned int *bad, hipStream_t st)
{
    uint64_t *key_hi = (uint64_t *)scratch, *key_lo = key_hi + m, *s_hi = key_lo + m, *s_lo = s_hi + m;
    unsigned long long *cnt_hi = (unsigned long long *)(s_lo + m), *cnt_lo = cnt_hi + (n + 1);
    uint64_t *off_hi = (uint64_t *)(cnt_lo + (n + 1)), *off_lo = off_hi + (n + 1);
    hipError_t e;
    launch_fill_u64((uint64_t *)cnt_hi, 0, 2 * (n + 1), st);
    launch_fill_u32(bad, 0u, 1, st);
    if (m > 0)
        hipLaunchKernelGGL(csr_keys_kernel, dim3(grid_for(m)), dim3(256), 0, st, pairs, m, n, key_hi, key_lo, cnt_hi,
                           cnt_lo, bad);
    size_t tb = sort_bytes;
    if (m > 0) {
        if ((e = rocprim::radix_sort_keys(sort_tmp, tb, (const uint64_t *)key_hi, s_hi, (unsigned int)m, 0, 64, st)))
            return e;
        tb = sort_bytes;
        if ((e = rocprim::radix_sort_keys(sort_tmp, tb, (const uint64_t *)key_lo, s_lo, (unsigned int)m, 0, 64, st)))
            return e;
    }
    tb = sort_bytes;
    if ((e = rocprim::exclusive_scan(sort_tmp, tb, (const uint64_t *)cnt_hi, off_hi, (uint64_t)0, (size_t)(n + 1),
                                     rocprim::plus<uint64_t>(), st)))
        return e;
    tb = sort_bytes;
    if ((e = rocprim::exclusive_scan(sort_tmp, tb, (const uint64_t *)cnt_lo, off_lo, (uint64_t)0, (size_t)(n + 1),
                                     rocprim::plus<uint64_t>(), st)))
        return e;
    hipLaunchKernelGGL(csr_rows_kernel, dim3(grid_for(n + 1)), dim3(256), 0, st, (const uint64_t *)off_lo,
                       (const uint64_t *)off_hi, n, row_ptr);
    if (m > 0) {
        hipLaunchKernelGGL(csr_fill_lo_kernel, dim3(grid_for(m)), dim3(256), 0, st, (const uint64_t *)s_lo, m,
                           (const uint64_t *)off_lo, (const int64_t *)row_ptr, cols);
        hipLaunchKernelGGL(csr_fill_hi_kernel, dim3(grid_for(m)), dim3(256), 0, st, (const uint64_t *)s_hi, m,
                           (const uint64_t *)off_hi, (const unsigned long long *)cnt_lo, (const int64_t *)row_ptr,
                           cols);
    }
    return hipGetLastError();
}

}  // namespace cpmi
