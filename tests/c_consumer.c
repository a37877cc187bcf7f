/* A plain C99 consumer of the library: the public headers compile as C and
 * the library links from C. It calls only what needs no GPU: argument checks
 * reject a null context and bad arguments. */
#include <stdio.h>

#include "cpmi.h"
#include "cpmi_debug.h"

int main(void)
{
    cpmi_pair best;
    cpmi_match_pair mp;
    int64_t count = 0, pairs = 0;
    int bad = 0;
    bad |= cpmi_closest_pair(NULL, NULL, CPMI_F32, 10, 4, 4, CPMI_PREC_AUTO, NULL, &best) != CPMI_ERR_ARG;
    bad |= cpmi_frnn(NULL, NULL, CPMI_F32, 10, 4, 4, 1.0, CPMI_PREC_BF16, NULL, NULL, NULL, 0, &count) != CPMI_ERR_ARG;
    bad |= cpmi_motif(NULL, NULL, 100, 8, 0, CPMI_PREC_AUTO, -1.0, NULL, &best, NULL, NULL, 0, NULL) != CPMI_ERR_ARG;
    bad |= cpmi_strings_pair(NULL, NULL, 10, 4, 4, 3, CPMI_MOST_CORRELATED, NULL, &mp) != CPMI_ERR_ARG;
    bad |= cpmi_two_locus(NULL, NULL, 5, 5, 10, 10, 0, NULL, &mp) != CPMI_ERR_ARG;
    bad |= cpmi_strings_lightbulb(NULL, NULL, 10, 4, 4, 3, 0, 1, 2, 0, 16, NULL, &mp, &pairs) != CPMI_ERR_ARG;
    bad |= cpmi_set_pruning(NULL, 1, 10.0, 0) != CPMI_ERR_ARG;
    bad |= cpmi_pairs_to_csr(NULL, NULL, 0, 10, NULL, NULL, NULL) != CPMI_ERR_ARG;
    bad |= cpmi_closest_pair_noalloc(NULL, NULL, CPMI_F32, 10, 4, 4, CPMI_PREC_AUTO, NULL, &best) != CPMI_ERR_ARG;
    bad |= cpmi_dbg_set_prune_order(NULL, 0, 1.0) != CPMI_ERR_ARG;
    bad |= cpmi_dbg_tile_list(10, 0, 128, NULL, 0) != CPMI_ERR_ARG;
    bad |= cpmi_version() != 10000;
    printf("%s\n", bad ? "FAIL" : "ok");
    return bad;
}
