// Randomised light-bulb bucketing (Section 4, MLBA; Section 5 for the least
// correlated pair) as a candidate generator on the GPU.
//
// One iteration: a key per row from the symbols (bits) of c randomly chosen
// columns, a radix sort of the rows by key, every pair of rows that share a
// bucket (equal keys) added to the candidates, and the candidates' exact
// match counts merged into the best pair so far. The iterations run in
// batches: one key kernel, one sort (keys tagged with their iteration, or a
// segment per iteration where the tag does not fit in 64 bits), a counting
// pass over the buckets and a prefix sum of its counts, then a pass that
// writes the candidates at their offsets and one verification of them all.
// After enough iterations the best pair is the most (least) correlated one
// with high probability; the reported count is always the pair's exact one.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>

#include "cpmi_internal.h"

namespace cpmi {

namespace {

// Key of row r in iteration b of the batch (blockIdx.y): the chosen
// columns' values, bits_per packed bits each, first column in the most
// significant place. Rows are strings (mode 0: symbols, bits_per =
// ceil(log2 sigma)) or the one-hot bit strings of Section 5 (mode 1: the
// codes of the n strings, then their complements; a column is a bit position
// c * sigma + b of the codes, set where S[c] == sigma - 1 - b). With tag
// set, the iteration's index sits above the ncols * bits_per key bits, so
// that one sort of the whole batch keeps the iterations apart.
__global__ void lb_keys_kernel(const signed char *S, int64_t n, int64_t ld, int sigma, int mode, int bits_per,
                               const int32_t *cols_all, int ncols, bool tag, uint64_t *keys_all, int32_t *rows_all)
{
    const int64_t total = mode == 0 ? n : 2 * n;
    const int b = blockIdx.y;
    const int32_t *cols = cols_all + (int64_t)b * ncols;
    uint64_t *keys = keys_all + (int64_t)b * total;
    int32_t *rows = rows_all + (int64_t)b * total;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < total; r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = r < n ? r : r - n;
        const bool comp = r >= n;
        uint64_t key = 0;
        for (int c = 0; c < ncols; ++c) {
            uint64_t v;
            if (mode == 0) {
                v = (uint64_t)(unsigned char)S[i * ld + cols[c]];
            } else {
                // bit b of symbol c's group is set for symbol sigma - 1 - b
                // (Section 5's order, 0 -> 0..01)
                const int32_t pos = cols[c];
                const int bit = S[i * ld + pos / sigma] == sigma - 1 - pos % sigma;
                v = (uint64_t)(comp ? !bit : bit);
            }
            key = (key << bits_per) | v;
        }
        keys[r] = tag ? key | ((uint64_t)b << (ncols * bits_per)) : key;
        rows[r] = (int32_t)r;
    }
}

// Every pair of a bucket (a run of equal keys in the sorted segment of its
// iteration): the thread of sorted position p pairs it with the positions
// after it in the run. Mode 1 keeps only (code, complement) pairs of
// different strings. Without cand, num[p] = the number of such pairs of p;
// with it, they are written to cand[off[p] - base ...] (off: the exclusive
// prefix sum of num over the batch), for the positions [p0, p1). Both passes
// take the same pairs in the same order; no atomics.
__global__ void lb_pairs_kernel(const uint64_t *keys, const int32_t *rows, int64_t total, int64_t p0, int64_t p1,
                                int64_t n, int mode, uint64_t *num, int2 *cand, const uint64_t *off, uint64_t base)
{
    for (int64_t p = p0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < p1;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t end = (p / total + 1) * total;
        const uint64_t kp = keys[p];
        uint64_t at = cand ? off[p] - base : 0, mine = 0;
        for (int64_t q = p + 1; q < end && keys[q] == kp; ++q) {
            int32_t a = rows[p], c = rows[q];
            if (mode == 1) {
                if ((a < n) == (c < n)) continue;                 // both codes or both complements
                if (a >= n) {
                    const int32_t t = a;
                    a = c;
                    c = t;
                }
                c -= (int32_t)n;                                   // complement of string c
                if (a == c) continue;
            }
            if (cand) cand[at++] = make_int2(a < c ? a : c, a < c ? c : a);
            else ++mine;
        }
        if (!cand) num[p] = mine;
    }
}

// Pairs of each iteration b < nb of the batch from the prefix sums:
// seg[b] = off[(b+1) total] - off[b total] (the last one ending at
// off[all - 1] + num[all - 1]).
__global__ void lb_segments_kernel(const uint64_t *num, const uint64_t *off, int64_t total, int nb, uint64_t *seg)
{
    const int b = threadIdx.x;
    if (b >= nb) return;
    const int64_t all = total * nb;
    const uint64_t hi = b + 1 < nb ? off[(b + 1) * total] : off[all - 1] + num[all - 1];
    seg[b] = hi - off[(int64_t)b * total];
}

// Exact match count of each candidate, merged into the best pair:
// most correlated: max of (u << 42 | ~(i << 21 | j) & (2^42 - 1));
// least correlated: min of (u << 42 | i << 21 | j) (ties to the smallest (i, j)).
__global__ void lb_verify_kernel(const signed char *S, int64_t k, int64_t ld, int mode, const int2 *cand, uint64_t m,
                                 unsigned long long *best)
{
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

unsigned lb_grid(int64_t total)
{
    const int64_t g = (total + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 16384 ? 16384 : g));
}

}  // namespace

// Bits of the iteration tag of a batch of B (0 for B = 1), or -1 when the
// tag does not fit above the key bits (the sort then takes a segment per
// iteration).
int lb_tag_bits(int B, int key_bits)
{
    int t = 0;
    while ((1 << t) < B) ++t;
    return key_bits + t <= 64 ? t : -1;
}

void launch_lb_keys(const signed char *S, int64_t n, int64_t ld, int sigma, int mode, int bits_per,
                    const int32_t *cols, int ncols, int B, uint64_t *keys, int32_t *rows, hipStream_t st)
{
    const int64_t total = mode == 0 ? n : 2 * n;
    const bool tag = lb_tag_bits(B, ncols * bits_per) > 0;
    hipLaunchKernelGGL(lb_keys_kernel, dim3(lb_grid(total), (unsigned)B), dim3(256), 0, st, S, n, ld, sigma, mode,
                       bits_per, cols, ncols, tag, keys, rows);
}

hipError_t lb_sort(void *temp, size_t *temp_bytes, const uint64_t *keys_in, uint64_t *keys_out, const int32_t *rows_in,
                   int32_t *rows_out, int64_t total, int B, const int32_t *seg, int key_bits, hipStream_t st)
{
    const int t = lb_tag_bits(B, key_bits);
    if (t >= 0)
        return rocprim::radix_sort_pairs(temp, *temp_bytes, keys_in, keys_out, rows_in, rows_out,
                                         (unsigned int)(total * B), 0, key_bits + t, st);
    return rocprim::segmented_radix_sort_pairs(temp, *temp_bytes, keys_in, keys_out, rows_in, rows_out,
                                               (unsigned int)(total * B), (unsigned int)B, seg, seg + 1, 0, key_bits,
                                               st);
}

void launch_lb_count(const uint64_t *keys, const int32_t *rows, int64_t total, int B, int64_t n, int mode,
                     uint64_t *num, uint64_t *off, void *temp, size_t temp_bytes, uint64_t *seg, hipStream_t st)
{
    const int64_t all = total * B;
    hipLaunchKernelGGL(lb_pairs_kernel, dim3(lb_grid(all)), dim3(256), 0, st, keys, rows, total, (int64_t)0, all, n,
                       mode, num, (int2 *)nullptr, (const uint64_t *)nullptr, (uint64_t)0);
    size_t tb = temp_bytes;
    rocprim::exclusive_scan(temp, tb, num, off, (uint64_t)0, (size_t)all, rocprim::plus<uint64_t>(), st);
    hipLaunchKernelGGL(lb_segments_kernel, dim3(1), dim3(256), 0, st, num, off, total, B, seg);
}

size_t lb_scan_bytes(int64_t all)
{
    size_t tb = 0;
    rocprim::exclusive_scan(nullptr, tb, (const uint64_t *)nullptr, (uint64_t *)nullptr, (uint64_t)0, (size_t)all,
                            rocprim::plus<uint64_t>(), (hipStream_t)0);
    return tb;
}

void launch_lb_fill(const uint64_t *keys, const int32_t *rows, int64_t total, int64_t p0, int64_t p1, int64_t n,
                    int mode, const uint64_t *off, uint64_t base, int2 *cand, hipStream_t st)
{
    if (p1 <= p0) return;
    hipLaunchKernelGGL(lb_pairs_kernel, dim3(lb_grid(p1 - p0)), dim3(256), 0, st, keys, rows, total, p0, p1, n, mode,
                       (uint64_t *)nullptr, cand, off, base);
}

void launch_lb_verify(const signed char *S, int64_t k, int64_t ld, int mode, const int2 *cand, uint64_t m,
                      unsigned long long *best, hipStream_t st)
{
    if (m == 0) return;
    hipLaunchKernelGGL(lb_verify_kernel, dim3(lb_grid((int64_t)std::min<uint64_t>(m, 1u << 22))), dim3(256), 0, st, S,
                       k, ld, mode, cand, m, best);
}

}  // namespace cpmi
