/* Drives the library's host side through its argument checks, its file
 * reading and its error reporting, up to the device query: built with the
 * address and undefined-behaviour sanitizers (host code only, no device code)
 * by test_sanitizers.py and run on a machine without a GPU.  Exits nonzero on
 * an unexpected status. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "../include/ising_search.h"

static int fails = 0;

static void expect(int got, int want, const char *what)
{
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, got, want, ising_search_last_error());
        ++fails;
    } else if (got != ISING_OK && strlen(ising_search_last_error()) == 0) {
        fprintf(stderr, "%s: no message for status %d\n", what, got);
        ++fails;
    }
}

int main(int argc, char **argv)
{
    const char *dir = argc > 1 ? argv[1] : ".";
    enum { N = 12, L = 2 };
    double J[N * N], h[N];
    uint64_t x[L];
    for (int i = 0; i < N; ++i) {
        h[i] = (double)((i * 37) % 11 - 5) / 1024.0;
        for (int j = 0; j < N; ++j) J[i * N + j] = i == j ? 0.0 : (double)(((i + 1) * (j + 1)) % 7 - 3) / 256.0;
    }
    x[0] = 0x5A5u;
    x[1] = 0x0F0u;
    const int32_t Ns[1] = {N};
    const double *Jp[1] = {J};
    const double *hp[1] = {h};
    const uint64_t *xp[1] = {x};
    ising_search_t *s = NULL;
    ising_config_t cfg;

    /* rejected before any device call */
    memset(&cfg, 0, sizeof cfg);
    cfg.M = 0;
    expect(ising_search_init(&s, &cfg, 1, Ns, Jp, hp, L, xp, NULL), ISING_ERR_INVALID_ARG, "M = 0");
    cfg.M = 4;
    cfg.flags = 1 << 20;
    expect(ising_search_init(&s, &cfg, 1, Ns, Jp, hp, L, xp, NULL), ISING_ERR_INVALID_ARG, "unknown flag");
    cfg.flags = 0;
    cfg.surv_capacity = 3;
    expect(ising_search_init(&s, &cfg, 1, Ns, Jp, hp, L, xp, NULL), ISING_ERR_INVALID_ARG, "surv_capacity");
    cfg.surv_capacity = 0;
    J[1] += 1.0 / 16777216.0;
    expect(ising_search_init(&s, &cfg, 1, Ns, Jp, hp, L, xp, NULL), ISING_ERR_INVALID_ARG, "asymmetric J");
    J[1] -= 1.0 / 16777216.0;
    x[0] |= (uint64_t)1 << 40;
    expect(ising_search_init(&s, &cfg, 1, Ns, Jp, hp, L, xp, NULL), ISING_ERR_INVALID_ARG, "stray bits");
    x[0] &= ~((uint64_t)1 << 40);
    expect(ising_search_init(NULL, &cfg, 1, Ns, Jp, hp, L, xp, NULL), ISING_ERR_INVALID_ARG, "NULL out");
    expect(ising_search_init(&s, NULL, 1, Ns, Jp, hp, L, xp, NULL), ISING_ERR_INVALID_ARG, "NULL cfg");

    /* the weights file: missing, short, then a good one */
    char wpath[4096], cpath[4096];
    snprintf(wpath, sizeof wpath, "%s/w.bin", dir);
    snprintf(cpath, sizeof cpath, "%s/tiles.txt", dir);
    cfg.form = ISING_FORM_LEARNED;
    cfg.mlp_weights = wpath;
    remove(wpath);
    expect(ising_search_init(&s, &cfg, 1, Ns, Jp, hp, L, xp, NULL), ISING_ERR_INVALID_ARG, "missing weights");
    const int np = ising_mlp_num_params();
    float *w = (float *)calloc((size_t)np + 1, sizeof(float));
    FILE *f = fopen(wpath, "wb");
    fwrite(w, sizeof(float), (size_t)np - 1, f);
    fclose(f);
    expect(ising_search_init(&s, &cfg, 1, Ns, Jp, hp, L, xp, NULL), ISING_ERR_INVALID_ARG, "short weights");
    f = fopen(wpath, "wb");
    fwrite(w, sizeof(float), (size_t)np, f);
    fclose(f);
    free(w);
    cfg.tile_cache = cpath;
    const int rc = ising_search_init(&s, &cfg, 1, Ns, Jp, hp, L, xp, NULL);
    if (rc == ISING_OK) ising_search_destroy(s);
    else expect(rc, ISING_ERR_NO_DEVICE, "good files");

    /* other entry points' checks */
    expect(ising_search_step(NULL, NULL), ISING_ERR_BAD_STATE, "step on NULL");
    ising_search_destroy(NULL);
    int32_t cnt = 0;
    expect(ising_brute_lowest(0, NULL, NULL, NULL, 1, NULL, NULL, NULL, NULL), ISING_ERR_INVALID_ARG, "brute, no instances");
    (void)cnt;
    printf("%d unexpected\n", fails);
    return fails != 0;
}
