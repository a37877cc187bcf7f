/* Drives the host-only logic of the cpmi library (tile lists, two-set lists,
 * pruned tile lists, tune-cache parsing and saving, bounds, layouts) for the
 * sanitizer build of the host code. No device work. Exit status 0 and "ok".
 * argv[1]: a scratch directory for tune-cache files. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "cpmi.h"
#include "cpmi_debug.h"

#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                              \
        }                                                          \
    } while (0)

static int write_file(const char *path, const char *text)
{
    FILE *f = fopen(path, "w");
    if (!f) return 0;
    fputs(text, f);
    fclose(f);
    return 1;
}

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    static uint64_t buf[1 << 16];
    /* tile lists over edges, exclusions and ragged sizes (count, then a short buffer) */
    const int64_t ns[] = {2, 255, 256, 257, 1000, 4097};
    const int64_t ex[] = {1, 3, 256, 300};
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 4; ++b)
            for (int t = 128; t <= 256; t += 128) {
                const int64_t cnt = cpmi_dbg_tile_list(ns[a], ex[b], t, buf, 1 << 16);
                CHECK(cnt >= 0);
                CHECK(cpmi_dbg_tile_list(ns[a], ex[b], t, buf, cnt > 2 ? 2 : cnt) == cnt);
            }
    CHECK(cpmi_dbg_tile_list(1000, 1, 100, buf, 10) < 0);
    int64_t nfull = 0;
    CHECK(cpmi_dbg_tile_list_two(300, 200, 512, 256, buf, 1 << 16, &nfull) >= 0);
    CHECK(cpmi_dbg_tile_list_two(1, 1, 256, 256, buf, 0, NULL) >= 0);
    CHECK(cpmi_dbg_tile_list_two(300, 200, 100, 256, buf, 10, NULL) < 0);   /* split not a multiple of 256 */
    /* pruned lists: intervals sorted by reference 0 */
    enum { NT = 40, Q = 3 };
    static double lo[NT * Q], hi[NT * Q];
    for (int I = 0; I < NT; ++I)
        for (int k = 0; k < Q; ++k) {
            lo[I * Q + k] = k == 0 ? 2.0 * I : 5.0 + ((I * 7 + k) % 11);
            hi[I * Q + k] = lo[I * Q + k] + (k == 0 ? 1.5 : 3.0);
        }
    int64_t np = 0;
    const double Ts[] = {-1.0, 0.0, 0.7, 3.0, 1e9};
    for (int t = 0; t < 5; ++t)
        for (int band = -1; band <= 2; ++band) {
            const int64_t cnt = cpmi_dbg_pruned_tiles(NT * 256 - 13, 256, Q, lo, hi, Ts[t], band, buf, 1 << 16,
                                                      &nfull, &np);
            CHECK(cnt >= 0 && nfull <= cnt);
            CHECK(cpmi_dbg_pruned_tiles(NT * 256 - 13, 256, Q, lo, hi, Ts[t], band, buf, 1, NULL, NULL) == cnt);
        }
    CHECK(cpmi_dbg_pruned_tiles(100, 256, 0, lo, hi, 1.0, -1, buf, 10, NULL, NULL) < 0);
    /* tune cache: good, malformed and truncated files, saved and read back */
    char in[1024], out[1024];
    int32_t p = 0, tl = 0;
    snprintf(in, sizeof in, "%s/good.json", argv[1]);
    snprintf(out, sizeof out, "%s/saved.json", argv[1]);
    CHECK(write_file(in, "{\n \"bf16:k512:r18\": 128,\n \"auto:k64:r12\": 1,\n \"i8:k4096:r17\": 256,\n \"band.bf16:k512:r18\": 16,\n \"band.auto:k64:r3\": 4,\n \"band.i8:k4096:r17\": 99\n}\n"));
    CHECK(cpmi_dbg_tune(in, out, 256, CPMI_F32, CPMI_PREC_BF16, 512, 3.4e10, &p, &tl) == CPMI_OK);
    CHECK(cpmi_dbg_tune(out, NULL, 256, CPMI_F32, CPMI_PREC_AUTO, 40, 1e6, &p, &tl) == CPMI_OK);
    const char *bad[] = {"", "{", "{\"bf16:k512:r18\": }", "{\"x:y\": 3}", "{\"bf16:k99999999999999999999:r3\": 128}",
                         "{\"bf16:k512:r18\": 12345678901234567890}", "not json at all", "{\"bf16:k512"};
    for (int i = 0; i < 8; ++i) {
        snprintf(in, sizeof in, "%s/bad%d.json", argv[1], i);
        CHECK(write_file(in, bad[i]));
        CHECK(cpmi_dbg_tune(in, out, 256, CPMI_F32, CPMI_PREC_AUTO, 512, 1e9, &p, &tl) == CPMI_OK);
    }
    CHECK(cpmi_dbg_tune("/nonexistent/dir/none.json", NULL, 8, CPMI_I8, CPMI_PREC_I8, 4096, 5e9, &p, &tl) ==
          CPMI_OK);
    /* bounds, layouts */
    const float bI[4] = {512.0f, 22.7f, 22.8f, 0.01f}, bJ[4] = {600.0f, 24.5f, 24.6f, 0.02f};
    CHECK(cpmi_dbg_tile_bound(bI, bJ, 512, 512, CPMI_PREC_BF16, 1) > 0.0);
    CHECK(cpmi_dbg_tile_bound(bI, bJ, 512, 500, CPMI_PREC_F32, 0) > 0.0);
    const double l1[2] = {0.0, 1.0}, h1[2] = {1.0, 2.0}, l2[2] = {5.0, 1.5}, h2[2] = {6.0, 1.6};
    CHECK(cpmi_dbg_tile_lb(l1, h1, l2, h2, 2) > 3.9);
    int32_t o4[4];
    for (int w = 0; w < 4; ++w)
        for (int q = 0; q < 4; ++q)
            for (int l = 0; l < 64; ++l) CHECK(cpmi_dbg_layout256(w, q, l, o4) == CPMI_OK);
    CHECK(cpmi_dbg_xs_offset256(300, 17, 1024) >= 0 && cpmi_dbg_xs_offset256(-1, 0, 1024) < 0);
    puts("ok");
    return 0;
}
