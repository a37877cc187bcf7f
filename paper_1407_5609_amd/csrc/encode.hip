// Encoders of the string problems into int8 rows for the matrix-core screen
// (Sections 5 and 6).
//
// A string over the alphabet {0, ..., sigma-1} becomes the concatenation of
// the one-hot codes of its symbols (symbol v -> sigma bits with bit v set; the
// paper's 0 -> 001, 1 -> 010, 2 -> 100 for sigma = 3, written here with bit v
// at offset v). Between two such codes the squared Euclidean distance of the
// 0/1 rows is their Hamming distance, 2 (k - u) for strings of length k that
// agree in u positions, so the least such distance is the most correlated
// pair. The complement of a code (every bit flipped) meets the code of an
// equal symbol in no bit and of a different symbol in two (the identity
// M(A'_i, ~A'_j) = 2 (k - u_ij) of Section 5): between a code row and a
// complemented row the squared distance is sigma k - 2 (k - u), least for the
// least correlated pair. For the two-locus problem (Section 6) the rows are
// the columns of D = [A' A'; B' ~B'] (or [A' ~A'; B' B'] for the opposite
// difference).
#include "cpmi_internal.h"

namespace cpmi {

namespace {

// Rows [0, n): codes of the strings; rows [split, split + n) (least
// correlated only): their complements. Rows [n, split) are zero. One thread
// per (string, position).
__global__ void encode_strings_kernel(const signed char *S, int64_t n, int64_t k, int64_t ld, int sigma,
                                      int complement, signed char *Z, int64_t Lz, int64_t split,
                                      unsigned int *flags)
{
    const int64_t total = n * k;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / k, c = t % k;
        const int s = S[i * ld + c];
        if (s < 0 || s >= sigma) atomicOr(flags, (unsigned int)F_SYMBOL);
        signed char *z = Z + i * Lz + (int64_t)sigma * c;
        for (int v = 0; v < sigma; ++v) z[v] = (signed char)(s == v);
        if (complement) {
            signed char *zc = Z + (split + i) * Lz + (int64_t)sigma * c;
            for (int v = 0; v < sigma; ++v) zc[v] = (signed char)(s != v);
        }
    }
}

// Two-locus rows from the genotype matrix G ((m1 + m2) x n, row s = subject
// s, the first m1 subjects cases): row i = column i of D's first half (codes
// of SNP i over cases then controls), row split + i = column n + i (codes
// over cases, complemented codes over controls; for direction 1 the cases'
// codes are complemented instead). A work-group transposes a tile of 64
// subjects x 64 SNPs through LDS: reads run along SNPs, writes along
// subjects.
__global__ __launch_bounds__(256) void encode_two_locus_kernel(const signed char *G, int64_t m1, int64_t m2,
                                                               int64_t n, int64_t ld, int direction, signed char *Z,
                                                               int64_t Lz, int64_t split, unsigned int *flags)
{
    __shared__ signed char tileT[64][65];
    const int64_t m = m1 + m2;
    const int64_t s0 = (int64_t)blockIdx.y * 64, i0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int64_t s = s0 + r, i = i0 + tx;
        signed char g = 0;
        if (s < m && i < n) {
            g = G[s * ld + i];
            if (g < 0 || g > 2) atomicOr(flags, (unsigned int)F_SYMBOL);
        }
        tileT[tx][r] = g;   // [SNP][subject]
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t i = i0 + r, s = s0 + tx;
        if (i >= n || s >= m) continue;
        const int g = tileT[r][tx];
        const bool flip = direction == 0 ? s >= m1 : s < m1;
        signed char *z = Z + i * Lz + 3 * s;
        signed char *zc = Z + (split + i) * Lz + 3 * s;
        for (int v = 0; v < 3; ++v) {
            z[v] = (signed char)(g == v);
            zc[v] = (signed char)(flip ? g != v : g == v);
        }
    }
}

// Flag F_SYMBOL if some symbol of the strings lies outside 0..sigma-1.
__global__ void check_symbols_kernel(const signed char *S, int64_t n, int64_t k, int64_t ld, int sigma,
                                     unsigned int *flags)
{
    const int64_t total = n * k;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int s = S[(t / k) * ld + t % k];
        if (s < 0 || s >= sigma) atomicOr(flags, (unsigned int)F_SYMBOL);
    }
}

unsigned grid_for(int64_t total)
{
    const int64_t g = (total + 255) / 256;
    return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace

void launch_encode_strings(const signed char *S, int64_t n, int64_t k, int64_t ld, int sigma, int complement,
                           signed char *Z, int64_t Lz, int64_t split, unsigned int *flags, hipStream_t st)
{
    hipLaunchKernelGGL(encode_strings_kernel, dim3(grid_for(n * k)), dim3(256), 0, st, S, n, k, ld, sigma, complement,
                       Z, Lz, split, flags);
}

void launch_check_symbols(const signed char *S, int64_t n, int64_t k, int64_t ld, int sigma, unsigned int *flags,
                          hipStream_t st)
{
    hipLaunchKernelGGL(check_symbols_kernel, dim3(grid_for(n * k)), dim3(256), 0, st, S, n, k, ld, sigma, flags);
}

void launch_encode_two_locus(const signed char *G, int64_t m1, int64_t m2, int64_t n, int64_t ld, int direction,
                             signed char *Z, int64_t Lz, int64_t split, unsigned int *flags, hipStream_t st)
{
    const dim3 g((unsigned)((n + 63) / 64), (unsigned)((m1 + m2 + 63) / 64));
    hipLaunchKernelGGL(encode_two_locus_kernel, g, dim3(256), 0, st, G, m1, m2, n, ld, direction, Z, Lz, split, flags);
}

}  // namespace cpmi
