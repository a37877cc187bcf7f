/* Drives the CPU oracle's entry points on small inputs, for the sanitizer
 * build (address and undefined-behaviour checks). Exit status 0 and "ok". */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_cpp_f32(const float *, int64_t, int64_t, int64_t, int64_t, int64_t *, int64_t *, double *);
int orc_cpp_f64(const double *, int64_t, int64_t, int64_t, int64_t, int64_t *, int64_t *, double *);
int orc_cpp_i8(const int8_t *, int64_t, int64_t, int64_t, int64_t, int64_t *, int64_t *, double *);
int orc_cpp_f64_lanes(const double *, int64_t, int64_t, int64_t, int64_t, int64_t *, int64_t *, double *);
int64_t orc_frnn_f32(const float *, int64_t, int64_t, int64_t, int64_t, double, int64_t *, double *, int64_t);
int64_t orc_frnn_i8(const int8_t *, int64_t, int64_t, int64_t, int64_t, double, int64_t *, double *, int64_t);
int64_t orc_frnn_f64_lanes(const double *, int64_t, int64_t, int64_t, int64_t, double, int64_t *, double *, int64_t);
int64_t orc_frnn_count_f32(const float *, int64_t, int64_t, int64_t, int64_t, double);
int orc_znorm(const float *, int64_t, int64_t, double *, double *, double *);
int orc_nn_f32(const float *, int64_t, int64_t, int64_t, double *);
void orc_block_d2_f32(const float *, int64_t, int64_t, int64_t, int64_t, int64_t, int64_t, double *);
int orc_strings_pair(const int8_t *, int64_t, int64_t, int64_t, int, int, int64_t *, int64_t *, int64_t *);
int orc_two_locus(const int8_t *, int64_t, int64_t, int64_t, int64_t, int, int64_t *, int64_t *, int64_t *);

static uint64_t st = 88172645463325252ull;
static double unif(void)
{
    st ^= st << 13;
    st ^= st >> 7;
    st ^= st << 17;
    return (double)(st >> 11) * 0x1p-53;
}

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                              \
        }                                                          \
    } while (0)

int main(void)
{
    enum { N = 203, D = 13, LD = 17 };
    float *X = malloc(sizeof(float) * N * LD);
    double *Xd = malloc(sizeof(double) * N * LD);
    int8_t *G = malloc((size_t)N * LD);
    for (int i = 0; i < N * LD; ++i) {
        X[i] = (float)(unif() * 4.0 - 2.0);
        Xd[i] = X[i];
        G[i] = (int8_t)(unif() * 3.0);
    }
    int64_t a, b, c;
    double v, w;
    CHECK(orc_cpp_f32(X, N, D, LD, 1, &a, &b, &v) == 0);
    CHECK(orc_cpp_f64(Xd, N, D, LD, 3, &a, &b, &v) == 0);
    CHECK(orc_cpp_f64_lanes(Xd, N, D, LD, 3, &c, &b, &w) == 0 && c == a && w == v);
    CHECK(orc_cpp_i8(G, N, D, LD, 1, &a, &b, &v) == 0);
    int64_t *pairs = malloc(sizeof(int64_t) * 2 * 4096);
    double *d2 = malloc(sizeof(double) * 4096);
    const int64_t m = orc_frnn_f32(X, N, D, LD, 1, 6.0, pairs, d2, 4096);
    CHECK(m > 0 && m <= 4096);
    CHECK(orc_frnn_count_f32(X, N, D, LD, 1, 6.0) == m);
    CHECK(orc_frnn_f64_lanes(Xd, N, D, LD, 1, 6.0, pairs, d2, 10) == m);   /* cap below the count */
    CHECK(orc_frnn_i8(G, N, D, LD, 2, 4.0, pairs, d2, 4096) >= 0);
    double *nn = malloc(sizeof(double) * N);
    CHECK(orc_nn_f32(X, N, D, LD, nn) == 0);
    double *blk = malloc(sizeof(double) * 20 * 31);
    orc_block_d2_f32(X, D, LD, 7, 20, 150, 31, blk);
    enum { L = 700, ELL = 37 };
    float *T = malloc(sizeof(float) * L);
    double acc = 0.0;
    for (int i = 0; i < L; ++i) T[i] = (float)(acc += unif() - 0.5);
    double *Xh = malloc(sizeof(double) * (L - ELL + 1) * ELL), *mu = malloc(sizeof(double) * L),
           *sg = malloc(sizeof(double) * L);
    CHECK(orc_znorm(T, L, ELL, Xh, mu, sg) == 0);
    CHECK(orc_cpp_f64_lanes(Xh, L - ELL + 1, ELL, ELL, ELL, &a, &b, &v) == 0);
    int8_t *S = malloc(60 * 9);
    for (int i = 0; i < 60 * 9; ++i) S[i] = (int8_t)(unif() * 4.0);
    CHECK(orc_strings_pair(S, 60, 9, 9, 4, 0, &a, &b, &c) == 0);
    CHECK(orc_strings_pair(S, 60, 9, 9, 4, 1, &a, &b, &c) == 0);
    int8_t *Gt = malloc(30 * 25);
    for (int i = 0; i < 30 * 25; ++i) Gt[i] = (int8_t)(unif() * 3.0);
    CHECK(orc_two_locus(Gt, 12, 18, 25, 25, 0, &a, &b, &c) == 0);
    CHECK(orc_two_locus(Gt, 12, 18, 25, 25, 1, &a, &b, &c) == 0);
    free(X), free(Xd), free(G), free(pairs), free(d2), free(nn), free(blk), free(T), free(Xh), free(mu), free(sg);
    free(S), free(Gt);
    puts("ok");
    return 0;
}
