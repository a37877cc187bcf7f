/*
 * CPU oracle for the exact closest-pair / fixed-radius-neighbour / motif path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library calls, links or
 * loads this file; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg do. It shares no code, header or constant with the GPU path.
 *
 * What it computes is the plain definition, by brute force:
 *
 *  - Distance (Section 2): d(x,y)^2 = sum_k (x_k - y_k)^2 over the l
 *    coordinates. The paper's straightforward algorithm evaluates it for every
 *    pair in O(l) each, O(n^2 l) in total (Section 3, opening paragraph).
 *  - Closest pair (Section 3, problem statement; MPR step 5 keeps the pair with
 *    the least distance): the pair i<j of least squared distance. Among exact
 *    ties the lexicographically smallest (i,j) is reported; iterating i then j
 *    in ascending order with a strict "<" update yields exactly that pair.
 *  - Fixed-radius neighbours (Section 3.5, MPR-FRNNS step 5): every pair i<j
 *    with d <= R, tested on squared values as d^2 <= R2 with R2 given by the
 *    caller. N(i) is the symmetric closure of this list.
 *  - Motif (Section 2 l-mers; Section 3): the windows T_i = a_i..a_{i+l-1} are
 *    z-normalised and a pair is admissible only when j - i >= excl (trivial
 *    matches of overlapping windows are excluded).
 *
 * Canonical arithmetic (makes "exact match" well defined; the GPU verifier is
 * written independently to the same rules):
 *  - float32 inputs are promoted exactly to double;
 *  - d^2 = acc with acc = 0 and, for k = 0..d-1 ascending, acc = fma(t,t,acc),
 *    t = x_ik - x_jk in double;
 *  - z-normalisation of window i: mu = (ascending double sum of T_{i+k}) / l;
 *    v = (ascending fma(e,e,.) with e = T_{i+k} - mu) / l (population
 *    variance, two passes); sigma = sqrt(v); xhat_k = (T_{i+k} - mu) / sigma.
 *  - int8 inputs: d^2 = sum_k (x_ik - x_jk)^2 in int64, exact.
 * Build with -ffp-contract=off and without fast-math so that every operation
 * is a single IEEE double operation rounded to nearest even.
 *
 * Indices are 0-based (the paper's are 1-based).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_NOPAIR (-2)
#define ORC_DEGENERATE (-4)
#define ORC_NOMEM (-8)

int orc_abi_version(void) { return 1; }

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* single-pair distances (Section 2)                                         */
/* ------------------------------------------------------------------------ */

double orc_d2_f32(const float *X, int64_t d, int64_t ld, int64_t i, int64_t j)
{
    const float *x = X + i * ld, *y = X + j * ld;
    double acc = 0.0;
    for (int64_t k = 0; k < d; ++k) {
        double t = (double)x[k] - (double)y[k];
        acc = fma(t, t, acc);
    }
    return acc;
}

double orc_d2_f64(const double *X, int64_t d, int64_t ld, int64_t i, int64_t j)
{
    const double *x = X + i * ld, *y = X + j * ld;
    double acc = 0.0;
    for (int64_t k = 0; k < d; ++k) {
        double t = x[k] - y[k];
        acc = fma(t, t, acc);
    }
    return acc;
}

int64_t orc_d2_i8(const int8_t *X, int64_t d, int64_t ld, int64_t i, int64_t j)
{
    const int8_t *x = X + i * ld, *y = X + j * ld;
    int64_t acc = 0;
    for (int64_t k = 0; k < d; ++k) {
        int64_t t = (int64_t)x[k] - (int64_t)y[k];
        acc += t * t;
    }
    return acc;
}

/* d^2 from row i to every row j (out[i] = 0). Used for sampled checks. */
void orc_row_d2_f32(const float *X, int64_t n, int64_t d, int64_t ld, int64_t i, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) out[j] = orc_d2_f32(X, d, ld, i, j);
}

void orc_row_d2_f64(const double *X, int64_t n, int64_t d, int64_t ld, int64_t i, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) out[j] = orc_d2_f64(X, d, ld, i, j);
}

void orc_row_d2_i8(const int8_t *X, int64_t n, int64_t d, int64_t ld, int64_t i, int64_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) out[j] = orc_d2_i8(X, d, ld, i, j);
}

/* ------------------------------------------------------------------------ */
/* z-normalised l-mers (Section 2 defines the l-mers; normalisation is the    */
/* motif-mining convention, canonical two-pass population form above)        */
/* ------------------------------------------------------------------------ */

int orc_znorm(const float *T, int64_t len, int64_t ell, double *Xhat, double *mu_out, double *sigma_out)
{
    if (ell < 1 || len < ell) return ORC_NOPAIR;
    int64_t N = len - ell + 1;
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int64_t i = 0; i < N; ++i) {
        double s = 0.0;
        for (int64_t k = 0; k < ell; ++k) s += (double)T[i + k];
        double mu = s / (double)ell;
        double v = 0.0;
        for (int64_t k = 0; k < ell; ++k) {
            double e = (double)T[i + k] - mu;
            v = fma(e, e, v);
        }
        v = v / (double)ell;
        double sigma = sqrt(v);
        if (mu_out) mu_out[i] = mu;
        if (sigma_out) sigma_out[i] = sigma;
        if (!(sigma > 0.0)) { bad = 1; continue; }
        if (Xhat)
            for (int64_t k = 0; k < ell; ++k) Xhat[i * ell + k] = ((double)T[i + k] - mu) / sigma;
    }
    return bad ? ORC_DEGENERATE : ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* closest pair (Section 3 problem; MPR step 5 update rule)                  */
/* ------------------------------------------------------------------------ */

/* Lexicographic order on (d2, i, j). */
static int better(double d2a, int64_t ia, int64_t ja, double d2b, int64_t ib, int64_t jb)
{
    if (d2a != d2b) return d2a < d2b;
    if (ia != ib) return ia < ib;
    return ja < jb;
}

#define ORC_CPP_BODY(D2EXPR)                                                     \
    double best = INFINITY;                                                      \
    int64_t bi = -1, bj = -1;                                                    \
    _Pragma("omp parallel")                                                      \
    {                                                                            \
        double tb = INFINITY;                                                    \
        int64_t ti = -1, tj = -1;                                                \
        _Pragma("omp for schedule(dynamic, 8) nowait")                           \
        for (int64_t i = 0; i < n; ++i) {                                        \
            for (int64_t j = i + excl; j < n; ++j) {                             \
                double v = (D2EXPR);                                             \
                if (ti < 0 || better(v, i, j, tb, ti, tj)) {                     \
                    tb = v; ti = i; tj = j;                                      \
                }                                                                \
            }                                                                    \
        }                                                                        \
        _Pragma("omp critical")                                                  \
        {                                                                        \
            if (ti >= 0 && (bi < 0 || better(tb, ti, tj, best, bi, bj))) {      \
                best = tb; bi = ti; bj = tj;                                     \
            }                                                                    \
        }                                                                        \
    }                                                                            \
    if (bi < 0) return ORC_NOPAIR;                                               \
    *out_i = bi; *out_j = bj; *out_d2 = best;                                    \
    return ORC_OK;

/* Every thread keeps the (d2, i, j)-lexicographic minimum of the pairs it
 * scans and the merge applies the same order, so the result does not depend on
 * how rows are shared among threads. */
int orc_cpp_f32(const float *X, int64_t n, int64_t d, int64_t ld, int64_t excl,
                int64_t *out_i, int64_t *out_j, double *out_d2)
{
    if (excl < 1) excl = 1;
    ORC_CPP_BODY(orc_d2_f32(X, d, ld, i, j))
}

int orc_cpp_f64(const double *X, int64_t n, int64_t d, int64_t ld, int64_t excl,
                int64_t *out_i, int64_t *out_j, double *out_d2)
{
    if (excl < 1) excl = 1;
    ORC_CPP_BODY(orc_d2_f64(X, d, ld, i, j))
}

int orc_cpp_i8(const int8_t *X, int64_t n, int64_t d, int64_t ld, int64_t excl,
               int64_t *out_i, int64_t *out_j, double *out_d2)
{
    if (excl < 1) excl = 1;
    ORC_CPP_BODY((double)orc_d2_i8(X, d, ld, i, j))
}

/* ------------------------------------------------------------------------ */
/* The same closest pair over FP64 rows, with SIMD lanes across pairs.        */
/*                                                                            */
/* Only the schedule differs from orc_cpp_f64: every pair (i, j) still gets   */
/* acc = 0, then acc = fma(t, t, acc) with t = x_ik - x_jk for k ascending,   */
/* one IEEE double operation each (the vector fma rounds once per lane, as    */
/* the scalar fma() does), and the same (d2, i, j) order picks the answer.    */
/* Lanes hold eight consecutive j; rows j are repacked into panels of eight   */
/* so that a lane's k-th value sits next to its neighbours'. Four rows i      */
/* share each panel load. Used to write expected values of large motif        */
/* batches in reasonable time; its results are tested equal to the plain     */
/* loop's bit for bit.                                                        */
/* ------------------------------------------------------------------------ */

#include <immintrin.h>

#define ORC_PJ 8   /* lanes (j) per panel */
#define ORC_PI 4   /* rows i per register block */
#define ORC_IB 64  /* rows i per work item */

int orc_cpp_f64_lanes(const double *X, int64_t n, int64_t d, int64_t ld, int64_t excl,
                      int64_t *out_i, int64_t *out_j, double *out_d2)
{
    if (excl < 1) excl = 1;
    if (n < 2 || d < 1) return ORC_NOPAIR;
    const int64_t nb = (n + ORC_PJ - 1) / ORC_PJ;
    const int64_t ni = (n + ORC_PI - 1) / ORC_PI * ORC_PI;
    /* panels: P[b][k][lane] = X[b*8 + lane][k]; rows past n are zero */
    double *P = (double *)aligned_alloc(64, (size_t)(nb * d * ORC_PJ) * sizeof(double));
    /* rows i, contiguous, padded to a multiple of four rows with zeros */
    double *A = (double *)malloc((size_t)(ni * d) * sizeof(double));
    if (!P || !A) { free(P); free(A); return ORC_NOMEM; }
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b)
        for (int64_t k = 0; k < d; ++k)
            for (int64_t l = 0; l < ORC_PJ; ++l) {
                const int64_t j = b * ORC_PJ + l;
                P[(b * d + k) * ORC_PJ + l] = j < n ? X[j * ld + k] : 0.0;
            }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ni; ++i)
        for (int64_t k = 0; k < d; ++k) A[i * d + k] = i < n ? X[i * ld + k] : 0.0;

    double best = INFINITY;
    int64_t bi = -1, bj = -1;
    const int64_t nblk = (n + ORC_IB - 1) / ORC_IB;
#pragma omp parallel
    {
        double tb = INFINITY;
        int64_t ti = -1, tj = -1;
        double out[ORC_PI][ORC_PJ];
#pragma omp for schedule(dynamic, 1) nowait
        for (int64_t blk = 0; blk < nblk; ++blk) {
            const int64_t i0 = blk * ORC_IB;
            const int64_t i1 = i0 + ORC_IB < ni ? i0 + ORC_IB : ni;
            if (i0 + excl >= n) continue;
            for (int64_t b = (i0 + excl) / ORC_PJ; b < nb; ++b) {
                const double *pb = P + b * d * ORC_PJ;
                for (int64_t i = i0; i < i1; i += ORC_PI) {
                    if (i >= n) break;
                    if (b * ORC_PJ + ORC_PJ - 1 < i + excl) continue; /* no lane admissible */
                    const double *a0 = A + i * d, *a1 = a0 + d, *a2 = a1 + d, *a3 = a2 + d;
                    __m256d c00 = _mm256_setzero_pd(), c01 = _mm256_setzero_pd();
                    __m256d c10 = _mm256_setzero_pd(), c11 = _mm256_setzero_pd();
                    __m256d c20 = _mm256_setzero_pd(), c21 = _mm256_setzero_pd();
                    __m256d c30 = _mm256_setzero_pd(), c31 = _mm256_setzero_pd();
                    for (int64_t k = 0; k < d; ++k) {
                        const __m256d y0 = _mm256_load_pd(pb + k * ORC_PJ);
                        const __m256d y1 = _mm256_load_pd(pb + k * ORC_PJ + 4);
                        __m256d x, t;
                        x = _mm256_broadcast_sd(a0 + k);
                        t = _mm256_sub_pd(x, y0); c00 = _mm256_fmadd_pd(t, t, c00);
                        t = _mm256_sub_pd(x, y1); c01 = _mm256_fmadd_pd(t, t, c01);
                        x = _mm256_broadcast_sd(a1 + k);
                        t = _mm256_sub_pd(x, y0); c10 = _mm256_fmadd_pd(t, t, c10);
                        t = _mm256_sub_pd(x, y1); c11 = _mm256_fmadd_pd(t, t, c11);
                        x = _mm256_broadcast_sd(a2 + k);
                        t = _mm256_sub_pd(x, y0); c20 = _mm256_fmadd_pd(t, t, c20);
                        t = _mm256_sub_pd(x, y1); c21 = _mm256_fmadd_pd(t, t, c21);
                        x = _mm256_broadcast_sd(a3 + k);
                        t = _mm256_sub_pd(x, y0); c30 = _mm256_fmadd_pd(t, t, c30);
                        t = _mm256_sub_pd(x, y1); c31 = _mm256_fmadd_pd(t, t, c31);
                    }
                    _mm256_storeu_pd(out[0], c00); _mm256_storeu_pd(out[0] + 4, c01);
                    _mm256_storeu_pd(out[1], c10); _mm256_storeu_pd(out[1] + 4, c11);
                    _mm256_storeu_pd(out[2], c20); _mm256_storeu_pd(out[2] + 4, c21);
                    _mm256_storeu_pd(out[3], c30); _mm256_storeu_pd(out[3] + 4, c31);
                    for (int r = 0; r < ORC_PI; ++r)
                        for (int l = 0; l < ORC_PJ; ++l) {
                            const int64_t ii = i + r, jj = b * ORC_PJ + l;
                            if (ii >= n || jj >= n || jj < ii + excl) continue;
                            if (ti < 0 || better(out[r][l], ii, jj, tb, ti, tj)) {
                                tb = out[r][l]; ti = ii; tj = jj;
                            }
                        }
                }
            }
        }
#pragma omp critical
        {
            if (ti >= 0 && (bi < 0 || better(tb, ti, tj, best, bi, bj))) {
                best = tb; bi = ti; bj = tj;
            }
        }
    }
    free(P);
    free(A);
    if (bi < 0) return ORC_NOPAIR;
    *out_i = bi; *out_j = bj; *out_d2 = best;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* fixed-radius neighbours (Section 3.5, MPR-FRNNS emission d <= R)          */
/* ------------------------------------------------------------------------ */

typedef struct { int64_t i, j; double d2; } orc_rec;

static int rec_cmp(const void *a, const void *b)
{
    const orc_rec *x = (const orc_rec *)a, *y = (const orc_rec *)b;
    if (x->i != y->i) return x->i < y->i ? -1 : 1;
    if (x->j != y->j) return x->j < y->j ? -1 : 1;
    return 0;
}

typedef struct { orc_rec *v; int64_t n, cap; int fail; } orc_vec;

static void vec_push(orc_vec *a, int64_t i, int64_t j, double d2)
{
    if (a->fail) return;
    if (a->n == a->cap) {
        int64_t nc = a->cap ? a->cap * 2 : 1024;
        orc_rec *p = (orc_rec *)realloc(a->v, (size_t)nc * sizeof(orc_rec));
        if (!p) { a->fail = 1; return; }
        a->v = p; a->cap = nc;
    }
    a->v[a->n].i = i; a->v[a->n].j = j; a->v[a->n].d2 = d2; a->n++;
}

/* Returns the number of pairs (or a negative error). The first min(count, cap)
 * pairs in (i,j) order are written to pairs (2 int64 per pair) and d2. */
#define ORC_FRNN_BODY(D2EXPR)                                                    \
    orc_vec all = {0, 0, 0, 0};                                                  \
    _Pragma("omp parallel")                                                      \
    {                                                                            \
        orc_vec loc = {0, 0, 0, 0};                                              \
        _Pragma("omp for schedule(dynamic, 8) nowait")                           \
        for (int64_t i = 0; i < n; ++i)                                          \
            for (int64_t j = i + excl; j < n; ++j) {                             \
                double v = (D2EXPR);                                             \
                if (v <= R2) vec_push(&loc, i, j, v);                            \
            }                                                                    \
        _Pragma("omp critical")                                                  \
        {                                                                        \
            if (loc.fail) all.fail = 1;                                          \
            for (int64_t t = 0; t < loc.n; ++t)                                  \
                vec_push(&all, loc.v[t].i, loc.v[t].j, loc.v[t].d2);             \
        }                                                                        \
        free(loc.v);                                                             \
    }                                                                            \
    if (all.fail) { free(all.v); return ORC_NOMEM; }                             \
    if (all.n > 1) qsort(all.v, (size_t)all.n, sizeof(orc_rec), rec_cmp);        \
    for (int64_t t = 0; t < all.n && t < cap; ++t) {                             \
        pairs[2 * t] = all.v[t].i; pairs[2 * t + 1] = all.v[t].j;                \
        if (d2_out) d2_out[t] = all.v[t].d2;                                     \
    }                                                                            \
    int64_t cnt = all.n;                                                         \
    free(all.v);                                                                 \
    return cnt;

int64_t orc_frnn_f32(const float *X, int64_t n, int64_t d, int64_t ld, int64_t excl, double R2,
                     int64_t *pairs, double *d2_out, int64_t cap)
{
    if (excl < 1) excl = 1;
    ORC_FRNN_BODY(orc_d2_f32(X, d, ld, i, j))
}

int64_t orc_frnn_f64(const double *X, int64_t n, int64_t d, int64_t ld, int64_t excl, double R2,
                     int64_t *pairs, double *d2_out, int64_t cap)
{
    if (excl < 1) excl = 1;
    ORC_FRNN_BODY(orc_d2_f64(X, d, ld, i, j))
}

int64_t orc_frnn_i8(const int8_t *X, int64_t n, int64_t d, int64_t ld, int64_t excl, double R2,
                    int64_t *pairs, double *d2_out, int64_t cap)
{
    if (excl < 1) excl = 1;
    ORC_FRNN_BODY((double)orc_d2_i8(X, d, ld, i, j))
}

/* The same radius list over FP64 rows with SIMD lanes across pairs j, as
 * orc_cpp_f64_lanes does for the closest pair: each pair's d^2 is the
 * ascending-k fma chain of orc_d2_f64, compared with R2 as in orc_frnn_f64,
 * and the list is sorted the same way, so the output is the same bit for bit.
 * Used to write expected radius lists of large inputs. */
int64_t orc_frnn_f64_lanes(const double *X, int64_t n, int64_t d, int64_t ld, int64_t excl, double R2,
                           int64_t *pairs, double *d2_out, int64_t cap)
{
    if (excl < 1) excl = 1;
    if (n < 2 || d < 1) return 0;
    const int64_t nb = (n + ORC_PJ - 1) / ORC_PJ;
    const int64_t ni = (n + ORC_PI - 1) / ORC_PI * ORC_PI;
    double *P = (double *)aligned_alloc(64, (size_t)(nb * d * ORC_PJ) * sizeof(double));
    double *A = (double *)malloc((size_t)(ni * d) * sizeof(double));
    if (!P || !A) { free(P); free(A); return ORC_NOMEM; }
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; ++b)
        for (int64_t k = 0; k < d; ++k)
            for (int64_t l = 0; l < ORC_PJ; ++l) {
                const int64_t j = b * ORC_PJ + l;
                P[(b * d + k) * ORC_PJ + l] = j < n ? X[j * ld + k] : 0.0;
            }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ni; ++i)
        for (int64_t k = 0; k < d; ++k) A[i * d + k] = i < n ? X[i * ld + k] : 0.0;

    orc_vec all = {0, 0, 0, 0};
    const int64_t nblk = (n + ORC_IB - 1) / ORC_IB;
#pragma omp parallel
    {
        orc_vec loc = {0, 0, 0, 0};
        double out[ORC_PI][ORC_PJ];
#pragma omp for schedule(dynamic, 1) nowait
        for (int64_t blk = 0; blk < nblk; ++blk) {
            const int64_t i0 = blk * ORC_IB;
            const int64_t i1 = i0 + ORC_IB < ni ? i0 + ORC_IB : ni;
            if (i0 + excl >= n) continue;
            for (int64_t b = (i0 + excl) / ORC_PJ; b < nb; ++b) {
                const double *pb = P + b * d * ORC_PJ;
                for (int64_t i = i0; i < i1; i += ORC_PI) {
                    if (i >= n) break;
                    if (b * ORC_PJ + ORC_PJ - 1 < i + excl) continue;
                    const double *a0 = A + i * d, *a1 = a0 + d, *a2 = a1 + d, *a3 = a2 + d;
                    __m256d c00 = _mm256_setzero_pd(), c01 = _mm256_setzero_pd();
                    __m256d c10 = _mm256_setzero_pd(), c11 = _mm256_setzero_pd();
                    __m256d c20 = _mm256_setzero_pd(), c21 = _mm256_setzero_pd();
                    __m256d c30 = _mm256_setzero_pd(), c31 = _mm256_setzero_pd();
                    for (int64_t k = 0; k < d; ++k) {
                        const __m256d y0 = _mm256_load_pd(pb + k * ORC_PJ);
                        const __m256d y1 = _mm256_load_pd(pb + k * ORC_PJ + 4);
                        __m256d x, t;
                        x = _mm256_broadcast_sd(a0 + k);
                        t = _mm256_sub_pd(x, y0); c00 = _mm256_fmadd_pd(t, t, c00);
                        t = _mm256_sub_pd(x, y1); c01 = _mm256_fmadd_pd(t, t, c01);
                        x = _mm256_broadcast_sd(a1 + k);
                        t = _mm256_sub_pd(x, y0); c10 = _mm256_fmadd_pd(t, t, c10);
                        t = _mm256_sub_pd(x, y1); c11 = _mm256_fmadd_pd(t, t, c11);
                        x = _mm256_broadcast_sd(a2 + k);
                        t = _mm256_sub_pd(x, y0); c20 = _mm256_fmadd_pd(t, t, c20);
                        t = _mm256_sub_pd(x, y1); c21 = _mm256_fmadd_pd(t, t, c21);
                        x = _mm256_broadcast_sd(a3 + k);
                        t = _mm256_sub_pd(x, y0); c30 = _mm256_fmadd_pd(t, t, c30);
                        t = _mm256_sub_pd(x, y1); c31 = _mm256_fmadd_pd(t, t, c31);
                    }
                    _mm256_storeu_pd(out[0], c00); _mm256_storeu_pd(out[0] + 4, c01);
                    _mm256_storeu_pd(out[1], c10); _mm256_storeu_pd(out[1] + 4, c11);
                    _mm256_storeu_pd(out[2], c20); _mm256_storeu_pd(out[2] + 4, c21);
                    _mm256_storeu_pd(out[3], c30); _mm256_storeu_pd(out[3] + 4, c31);
                    for (int r = 0; r < ORC_PI; ++r)
                        for (int l = 0; l < ORC_PJ; ++l) {
                            const int64_t ii = i + r, jj = b * ORC_PJ + l;
                            if (ii >= n || jj >= n || jj < ii + excl) continue;
                            if (out[r][l] <= R2) vec_push(&loc, ii, jj, out[r][l]);
                        }
                }
            }
        }
#pragma omp critical
        {
            if (loc.fail) all.fail = 1;
            for (int64_t t = 0; t < loc.n; ++t) vec_push(&all, loc.v[t].i, loc.v[t].j, loc.v[t].d2);
        }
        free(loc.v);
    }
    free(P);
    free(A);
    if (all.fail) { free(all.v); return ORC_NOMEM; }
    if (all.n > 1) qsort(all.v, (size_t)all.n, sizeof(orc_rec), rec_cmp);
    for (int64_t t = 0; t < all.n && t < cap; ++t) {
        pairs[2 * t] = all.v[t].i; pairs[2 * t + 1] = all.v[t].j;
        if (d2_out) d2_out[t] = all.v[t].d2;
    }
    const int64_t cnt = all.n;
    free(all.v);
    return cnt;
}

/* d^2 of every pair (i0 + a, j0 + b), a < ni, b < nj, into out[a * nj + b]:
 * a block of the distance matrix (used to check sampled screen values). */
void orc_block_d2_f32(const float *X, int64_t d, int64_t ld, int64_t i0, int64_t ni, int64_t j0, int64_t nj,
                      double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < ni; ++a)
        for (int64_t b = 0; b < nj; ++b) out[a * nj + b] = orc_d2_f32(X, d, ld, i0 + a, j0 + b);
}

void orc_block_d2_f64(const double *X, int64_t d, int64_t ld, int64_t i0, int64_t ni, int64_t j0, int64_t nj,
                      double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < ni; ++a)
        for (int64_t b = 0; b < nj; ++b) out[a * nj + b] = orc_d2_f64(X, d, ld, i0 + a, j0 + b);
}

void orc_block_d2_i8(const int8_t *X, int64_t d, int64_t ld, int64_t i0, int64_t ni, int64_t j0, int64_t nj,
                     double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < ni; ++a)
        for (int64_t b = 0; b < nj; ++b) out[a * nj + b] = (double)orc_d2_i8(X, d, ld, i0 + a, j0 + b);
}

/* Number of pairs i<j (j-i >= excl) with d^2 <= R2, without listing them
 * (Section 3.5's output size; |N(i)| summed over i is twice this). */
int64_t orc_frnn_count_f32(const float *X, int64_t n, int64_t d, int64_t ld, int64_t excl, double R2)
{
    if (excl < 1) excl = 1;
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + excl; j < n; ++j) total += orc_d2_f32(X, d, ld, i, j) <= R2;
    return total;
}

/* ------------------------------------------------------------------------ */
/* nearest-neighbour squared distance of every point (over all j != i).      */
/* Used only to derive a workload's radius from the data; each unordered     */
/* pair is evaluated once and updates both endpoints (d^2 is symmetric under */
/* the canonical arithmetic because t = x_i - x_j only changes sign).        */
/* ------------------------------------------------------------------------ */

int orc_nn_f32(const float *X, int64_t n, int64_t d, int64_t ld, double *nn_out)
{
    int nt = orc_max_threads();
    double *buf = (double *)malloc((size_t)nt * (size_t)n * sizeof(double));
    if (!buf) return ORC_NOMEM;
    for (int64_t t = 0; t < (int64_t)nt * n; ++t) buf[t] = INFINITY;
#pragma omp parallel
    {
#ifdef _OPENMP
        double *mine = buf + (int64_t)omp_get_thread_num() * n;
#else
        double *mine = buf;
#endif
#pragma omp for schedule(dynamic, 8)
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) {
                double v = orc_d2_f32(X, d, ld, i, j);
                if (v < mine[i]) mine[i] = v;
                if (v < mine[j]) mine[j] = v;
            }
    }
    for (int64_t i = 0; i < n; ++i) {
        double m = INFINITY;
        for (int t = 0; t < nt; ++t)
            if (buf[(int64_t)t * n + i] < m) m = buf[(int64_t)t * n + i];
        nn_out[i] = m;
    }
    free(buf);
    return ORC_OK;
}

/* ------------------------------------------------------------------------
 * Strings and correlation by matches (Sections 5 and 6).
 *
 *  - m(x, y) (Section 5 notation): the number of positions where two strings
 *    of equal length agree. Strings are rows of symbols 0..sigma-1 (int8).
 *    The correlation of strings i and j is m(S_i, S_j) / k. The most
 *    correlated pair is the one of least Hamming distance (the light-bulb
 *    problem statement of Section 4); by brute force over the definition.
 *  - The deterministic mapping of Section 5: symbol v -> sigma bits with one
 *    1, written as in the paper (0 -> 0..001, 1 -> 0..010, ...: the bit of
 *    symbol v is the (v+1)-th from the right); the complement flips every bit.
 *    M(X, Y) counts the equal bits of two bit strings.
 *  - Least correlated pair (Section 5): with D1 the codes A' and D2 their
 *    complements, the pair (a in D1, b in D2), a != b, whose bit strings agree
 *    the most, reported as (min(a,b), max(a,b)).
 *  - Two-locus association (Section 6): D = [A' A'; B' ~B'] (direction 0;
 *    direction 1 swaps which half is complemented: [A' ~A'; B' B']), with A'
 *    and B' the codes of the cases' and the controls' SNP columns; the pair
 *    of columns (i, n + j), i != j, with the most equal bits, reported as
 *    (min(i,j), max(i,j)).
 * Ties go to the lexicographically smallest reported (i, j).
 * ---------------------------------------------------------------------- */

int64_t orc_matches(const int8_t *S, int64_t k, int64_t ld, int64_t i, int64_t j)
{
    int64_t u = 0;
    for (int64_t c = 0; c < k; ++c) u += S[i * ld + c] == S[j * ld + c];
    return u;
}

void orc_encode(const int8_t *S, int64_t n, int64_t k, int64_t ld, int sigma, int complement, int8_t *X)
{
    const int64_t L = (int64_t)sigma * k;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t c = 0; c < k; ++c)
            for (int b = 0; b < sigma; ++b) {
                const int bit = S[i * ld + c] == sigma - 1 - b;   /* b counts from the left */
                X[i * L + c * sigma + b] = (int8_t)(complement ? 1 - bit : bit);
            }
}

int64_t orc_bit_matches(const int8_t *X, const int8_t *Y, int64_t L, int64_t i, int64_t j)
{
    int64_t m = 0;
    for (int64_t b = 0; b < L; ++b) m += X[i * L + b] == Y[j * L + b];
    return m;
}

/* Best pair under "more is better" over the pairs a != b of rows of X
 * (first set) and Y (second set) of L bits, reported unordered; or, with
 * Y == NULL, over the pairs a < b of X. */
static int best_bit_pair(const int8_t *X, const int8_t *Y, int64_t n, int64_t L, int64_t *oi, int64_t *oj,
                         int64_t *om)
{
    int64_t bi = -1, bj = -1, bm = -1;
#pragma omp parallel
    {
        int64_t ti = -1, tj = -1, tm = -1;
#pragma omp for schedule(dynamic, 4)
        for (int64_t a = 0; a < n; ++a) {
            for (int64_t b = Y ? 0 : a + 1; b < n; ++b) {
                if (a == b) continue;
                const int64_t m = orc_bit_matches(X, Y ? Y : X, L, a, b);
                const int64_t i = a < b ? a : b, j = a < b ? b : a;
                if (m > tm || (m == tm && (i < ti || (i == ti && j < tj)))) {
                    tm = m;
                    ti = i;
                    tj = j;
                }
            }
        }
#pragma omp critical
        {
            if (tm > bm || (tm == bm && tm >= 0 && (ti < bi || (ti == bi && tj < bj)))) {
                bm = tm;
                bi = ti;
                bj = tj;
            }
        }
    }
    if (bm < 0) return ORC_NOPAIR;
    *oi = bi;
    *oj = bj;
    *om = bm;
    return ORC_OK;
}

int orc_strings_pair(const int8_t *S, int64_t n, int64_t k, int64_t ld, int sigma, int mode, int64_t *oi,
                     int64_t *oj, int64_t *omatches)
{
    if (n < 2) return ORC_NOPAIR;
    if (mode == 0) {
        int64_t bi = -1, bj = -1, bu = -1;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t j = i + 1; j < n; ++j) {
                const int64_t u = orc_matches(S, k, ld, i, j);
                if (u > bu) {
                    bu = u;
                    bi = i;
                    bj = j;
                }
            }
        *oi = bi;
        *oj = bj;
        *omatches = bu;
        return ORC_OK;
    }
    const int64_t L = (int64_t)sigma * k;
    int8_t *A = (int8_t *)malloc((size_t)(n * L)), *Ac = (int8_t *)malloc((size_t)(n * L));
    if (!A || !Ac) {
        free(A);
        free(Ac);
        return ORC_NOMEM;
    }
    orc_encode(S, n, k, ld, sigma, 0, A);
    orc_encode(S, n, k, ld, sigma, 1, Ac);
    int64_t m = 0;
    const int rc = best_bit_pair(A, Ac, n, L, oi, oj, &m);
    free(A);
    free(Ac);
    if (rc == ORC_OK) *omatches = orc_matches(S, k, ld, *oi, *oj);
    return rc;
}

int orc_two_locus(const int8_t *G, int64_t m1, int64_t m2, int64_t n, int64_t ld, int direction, int64_t *oi,
                  int64_t *oj, int64_t *omatches)
{
    if (n < 2) return ORC_NOPAIR;
    const int64_t m = m1 + m2, L = 3 * m;
    /* rows of D1 and D2 are the columns of D: bits over subjects, cases first */
    int8_t *D1 = (int8_t *)malloc((size_t)(n * L)), *D2 = (int8_t *)malloc((size_t)(n * L));
    int8_t *col = (int8_t *)malloc((size_t)m);
    int8_t *code = (int8_t *)malloc((size_t)L), *comp = (int8_t *)malloc((size_t)L);
    if (!D1 || !D2 || !col || !code || !comp) {
        free(D1);
        free(D2);
        free(col);
        free(code);
        free(comp);
        return ORC_NOMEM;
    }
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t s = 0; s < m; ++s) col[s] = G[s * ld + i];
        orc_encode(col, 1, m, m, 3, 0, code);
        orc_encode(col, 1, m, m, 3, 1, comp);
        for (int64_t b = 0; b < L; ++b) {
            const int cases = b < 3 * m1;
            D1[i * L + b] = code[b];
            D2[i * L + b] = (direction == 0 ? !cases : cases) ? comp[b] : code[b];
        }
    }
    const int rc = best_bit_pair(D1, D2, n, L, oi, oj, omatches);
    free(D1);
    free(D2);
    free(col);
    free(code);
    free(comp);
    return rc;
}
