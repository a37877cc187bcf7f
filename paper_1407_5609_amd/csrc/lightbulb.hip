// Randomised light-bulb bucketing (Section 4, MLBA; Section 5 for the least
// correlated pair) as a candidate generator on the GPU.
//
// One iteration: a key per row from the symbols (bits) of c randomly chosen
// columns, a radix sort of the rows by key, every pair of rows that share a
// bucket (equal keys) added to the candidates, and the candidates' exact
// match counts merged into the best pair so far. After enough iterations the
// best pair is the most (least) correlated one with high probability; the
// reported count is always the pair's exact one.
#include <rocprim/device/device_radix_sort.hpp>

#include "cpmi_internal.h"

namespace cpmi {

namespace {

// Key of row r: the chosen columns' values, bits_per packed bits each, first
// column in the most significant place. Rows are strings (mode 0: symbols,
// bits_per = ceil(log2 sigma)) or the one-hot bit strings of Section 5 (mode
// 1: the codes of the n strings, then their complements; a column is a bit
// position c * sigma + b, bit b of the code of symbol S[c] being S[c] == b).
__global__ void lb_keys_kernel(const signed char *S, int64_t n, int64_t ld, int sigma, int mode, int bits_per,
                               const int32_t *cols, int ncols, uint64_t *keys, int32_t *rows)
{
    const int64_t total = mode == 0 ? n : 2 * n;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < total; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = r < n ? r : r - n;
        const bool comp = r >= n;
        uint64_t key = 0;
        for (int c = 0; c < ncols; ++c) {
            uint64_t v;
            if (mode == 0) {
                v = (uint64_t)(unsigned char)S[i * ld + cols[c]];
            } else {
                const int32_t pos = cols[c];
                const int bit = S[i * ld + pos / sigma] == pos % sigma;
                v = (uint64_t)(comp ? !bit : bit);
            }
            key = (key << bits_per) | v;
        }
        keys[r] = key;
        rows[r] = (int32_t)r;
    }
}

// Every pair of a bucket (a run of equal keys in sorted order): the thread of
// sorted position p pairs it with the positions after it in the run. Mode 1
// keeps only (code, complement) pairs of different strings. Candidates
// beyond `cap` are counted but not stored.
__global__ void lb_pairs_kernel(const uint64_t *keys, const int32_t *rows, int64_t total, int64_t n, int mode,
                                int2 *cand, uint32_t cap, unsigned long long *count)
{
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total; p += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t kp = keys[p];
        for (int64_t q = p + 1; q < total && keys[q] == kp; ++q) {
            int32_t a = rows[p], b = rows[q];
            if (mode == 1) {
                if ((a < n) == (b < n)) continue;                 // both codes or both complements
                if (a >= n) {
                    const int32_t t = a;
                    a = b;
                    b = t;
                }
                b -= (int32_t)n;                                   // complement of string b
                if (a == b) continue;
            }
            const int32_t i = a < b ? a : b, j = a < b ? b : a;
            const unsigned long long idx = atomicAdd(count, 1ull);
            if (idx < cap) cand[idx] = make_int2(i, j);
        }
    }
}

// Exact match count of each candidate, merged into the best pair:
// most correlated: max of (u << 42 | ~(i << 21 | j) & (2^42 - 1));
// least correlated: min of (u << 42 | i << 21 | j) (ties to the smallest (i, j)).
__global__ void lb_verify_kernel(const signed char *S, int64_t k, int64_t ld, int mode, const int2 *cand,
                                 const unsigned long long *count, uint32_t cap, unsigned long long *best)
{
    const uint64_t m = min<uint64_t>(*count, (uint64_t)cap);
    for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < m; c += (uint64_t)gridDim.x * blockDim.x) {
        const int2 pr = cand[c];
        const signed char *x = S + (int64_t)pr.x * ld, *y = S + (int64_t)pr.y * ld;
        uint64_t u = 0;
        for (int64_t t = 0; t < k; ++t) u += x[t] == y[t];
        const uint64_t ij = ((uint64_t)pr.x << 21) | (uint64_t)pr.y;
        if (mode == 0) atomicMax(best, (unsigned long long)((u << 42) | (~ij & ((1ull << 42) - 1))));
        else atomicMin(best, (unsigned long long)((u << 42) | ij));
    }
}

// After an iteration: add its candidate count to the running total and flag
// an overflow of the candidate buffer.
__global__ void lb_account_kernel(const unsigned long long *count, uint32_t cap, unsigned long long *total,
                                  unsigned int *overflow)
{
    total[0] += count[0];
    if (count[0] > cap) overflow[0] = 1u;
}

unsigned lb_grid(int64_t total)
{
    const int64_t g = (total + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

}  // namespace

void launch_lb_keys(const signed char *S, int64_t n, int64_t ld, int sigma, int mode, int bits_per,
                    const int32_t *cols, int ncols, uint64_t *keys, int32_t *rows, hipStream_t st)
{
    const int64_t total = mode == 0 ? n : 2 * n;
    hipLaunchKernelGGL(lb_keys_kernel, dim3(lb_grid(total)), dim3(256), 0, st, S, n, ld, sigma, mode, bits_per, cols,
                       ncols, keys, rows);
}

hipError_t lb_sort(void *temp, size_t *temp_bytes, const uint64_t *keys_in, uint64_t *keys_out, const int32_t *rows_in,
                   int32_t *rows_out, int64_t total, int key_bits, hipStream_t st)
{
    return rocprim::radix_sort_pairs(temp, *temp_bytes, keys_in, keys_out, rows_in, rows_out, (unsigned int)total, 0,
                                     key_bits, st);
}

void launch_lb_pairs(const uint64_t *keys, const int32_t *rows, int64_t total, int64_t n, int mode, int2 *cand,
                     uint32_t cap, unsigned long long *count, hipStream_t st)
{
    hipLaunchKernelGGL(lb_pairs_kernel, dim3(lb_grid(total)), dim3(256), 0, st, keys, rows, total, n, mode, cand, cap,
                       count);
}

void launch_lb_verify(const signed char *S, int64_t k, int64_t ld, int mode, const int2 *cand,
                      const unsigned long long *count, uint32_t cap, unsigned long long *best,
                      unsigned long long *total, unsigned int *overflow, hipStream_t st)
{
    hipLaunchKernelGGL(lb_verify_kernel, dim3(4096), dim3(256), 0, st, S, k, ld, mode, cand, count, cap, best);
    hipLaunchKernelGGL(lb_account_kernel, dim3(1), dim3(1), 0, st, count, cap, total, overflow);
}

}  // namespace cpmi
