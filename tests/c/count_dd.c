/* Plain C client of libtpcf.so: uploads a catalog read from stdin
 * ("n" then n lines "ra dec" in degrees) and "nbins" then nbins+1 edges,
 * counts DD with each precision and prints one line of nbins+2 counts per
 * precision.  Exits non-zero with the library's message on any error. */
#include <stdio.h>
#include <stdlib.h>

#include "tpcf.h"

static int check(int rc, const char *what) {
    if (rc != TPCF_OK) {
        fprintf(stderr, "%s failed (%d): %s\n", what, rc, tpcf_last_error(NULL));
        exit(1);
    }
    return rc;
}

int main(void) {
    long long n = 0;
    int nbins = 0;
    if (scanf("%lld", &n) != 1 || n < 0)
        return 2;
    double *ra = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    double *dec = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    for (long long i = 0; i < n; ++i)
        if (scanf("%lf %lf", &ra[i], &dec[i]) != 2)
            return 2;
    if (scanf("%d", &nbins) != 1 || nbins < 1)
        return 2;
    double *edges = (double *)malloc(sizeof(double) * (size_t)(nbins + 1));
    for (int k = 0; k <= nbins; ++k)
        if (scanf("%lf", &edges[k]) != 1)
            return 2;
    uint64_t *out = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nbins + 2));

    tpcf_ctx *ctx = NULL;
    check(tpcf_open(0, NULL, &ctx), "tpcf_open");
    int32_t cat = -1;
    check(tpcf_upload_catalog(ctx, ra, dec, (int64_t)n, &cat), "tpcf_upload_catalog");
    const int precisions[2] = {TPCF_FP32_CHORD, TPCF_FP64};
    for (int p = 0; p < 2; ++p) {
        check(tpcf_count(ctx, TPCF_DD, cat, -1, edges, nbins, precisions[p], -1, -1, out), "tpcf_count");
        for (int s = 0; s < nbins + 2; ++s)
            printf("%s%llu", s ? " " : "", (unsigned long long)out[s]);
        printf("\n");
    }
    /* an invalid request: DD with a second catalog */
    if (tpcf_count(ctx, TPCF_DD, cat, cat, edges, nbins, TPCF_FP32_CHORD, -1, -1, out) != TPCF_E_INVALID)
        return 3;
    check(tpcf_release_catalog(ctx, cat), "tpcf_release_catalog");
    check(tpcf_close(ctx), "tpcf_close");
    free(ra);
    free(dec);
    free(edges);
    free(out);
    return 0;
}
