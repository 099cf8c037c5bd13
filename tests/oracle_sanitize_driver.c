/*
 * Drives the CPU oracle (oracle/pa_oracle.c) through its public functions on
 * small graphs so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer checks every path: plain runs, noise levels,
 * both kinds of cluster move, adaptive steps, refused arguments, and the
 * helper functions. Test infrastructure (tests/test_sanitizers.py builds and
 * runs it); exits non-zero on a wrong return code, and the sanitizers abort
 * on any memory or undefined-behaviour error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_run(int32_t n, const int32_t *row_ptr, const int32_t *col, const int8_t *w, int32_t K,
               const double *beta, int32_t S, const int32_t *order, int32_t as_enable,
               int32_t as_stall_steps, int32_t as_max_level, int32_t as_frozen_inv, double as_gamma,
               int32_t nl_period, int32_t nl_kind, int32_t beta_adapt, int32_t adapt_jump,
               int32_t adapt_num, int32_t adapt_den, int32_t R, uint64_t seed, uint32_t inst,
               int32_t nthreads, int8_t *x_init, int8_t *x_out, int32_t *E_out, int64_t *best,
               int8_t *best_x, int64_t *stats, int32_t *counts);
int32_t oracle_icm_pair(int32_t n, const int32_t *row_ptr, const int32_t *col, int8_t *xa, int8_t *xb,
                        uint32_t draw, uint8_t *in_cluster);
uint64_t oracle_resample_counts(int32_t R, const uint64_t *W, uint64_t U, int32_t *n_out);

/* Symmetric CSR of a ring plus chords i -- i+7 (mod n), weights +-1 by index parity. */
static void graph(int n, int signed_w, int32_t **rp, int32_t **col, int8_t **w)
{
    int deg = n > 14 ? 4 : 2;
    *rp = malloc(sizeof(int32_t) * (size_t)(n + 1));
    *col = malloc(sizeof(int32_t) * (size_t)n * deg);
    *w = malloc((size_t)n * deg);
    int e = 0;
    for (int i = 0; i < n; ++i) {
        (*rp)[i] = e;
        int nb[4] = {(i + n - 1) % n, (i + 1) % n, (i + n - 7) % n, (i + 7) % n};
        for (int q = 0; q < deg; ++q) {
            int j = nb[q];
            int lo = i < j ? i : j, hi = i < j ? j : i;
            (*col)[e] = j;
            (*w)[e] = (signed_w && ((lo + hi) & 1)) ? -1 : 1;
            ++e;
        }
    }
    (*rp)[n] = e;
}

static int check(int got, int want, const char *what)
{
    if (got != want) {
        fprintf(stderr, "%s: returned %d, expected %d\n", what, got, want);
        return 1;
    }
    return 0;
}

int main(void)
{
    int bad = 0;
    for (int sg = 0; sg < 2; ++sg) {
        const int n = 40;
        int32_t *rp, *col;
        int8_t *w;
        graph(n, sg, &rp, &col, &w);
        double beta[12];
        for (int k = 0; k < 12; ++k) beta[k] = 0.1 + 0.2 * k;
        for (int variant = 0; variant < 5; ++variant) {
            int R = variant == 3 ? 7 : 24, K = 12;
            int as = variant >= 1, nl = variant == 2 || variant == 3 ? 2 : 0, kind = variant == 3;
            int adapt = variant == 4;
            int8_t *xi = malloc((size_t)R * n), *xo = malloc((size_t)R * n), *bx = malloc(n);
            int32_t *E = malloc(sizeof(int32_t) * R), *cnt = malloc(sizeof(int32_t) * (size_t)K * R);
            int64_t best[4], *st = malloc(sizeof(int64_t) * 10 * K);
            int rc = oracle_run(n, rp, col, w, K, beta, 3, NULL, as, 1, 4, 4, 0.8, nl, kind, adapt, 4, 1, 2,
                                R, 42 + variant, (uint32_t)variant, 2, xi, xo, E, best, bx, st, cnt);
            bad |= check(rc, 0, "oracle_run");
            free(xi); free(xo); free(bx); free(E); free(cnt); free(st);
        }
        /* refused arguments: decreasing beta, odd R with pair moves, uneven adaptive grid */
        double dec[3] = {0.5, 0.4, 0.6}, geo[4] = {0.1, 0.2, 0.4, 0.8};
        bad |= check(oracle_run(n, rp, col, w, 3, dec, 1, NULL, 0, 1, 4, 4, 0.8, 0, 0, 0, 4, 1, 2, 4, 1, 0, 1,
                                NULL, NULL, NULL, NULL, NULL, NULL, NULL), -1, "decreasing beta");
        bad |= check(oracle_run(n, rp, col, w, 3, beta, 1, NULL, 0, 1, 4, 4, 0.8, 2, 0, 0, 4, 1, 2, 5, 1, 0, 1,
                                NULL, NULL, NULL, NULL, NULL, NULL, NULL), -1, "odd R");
        bad |= check(oracle_run(n, rp, col, w, 4, geo, 1, NULL, 0, 1, 4, 4, 0.8, 0, 0, 1, 4, 1, 2, 4, 1, 0, 1,
                                NULL, NULL, NULL, NULL, NULL, NULL, NULL), -1, "uneven grid");
        /* a cluster move on two configurations */
        int8_t xa[40], xb[40];
        uint8_t mask[40];
        for (int i = 0; i < n; ++i) { xa[i] = (i % 3) ? 1 : -1; xb[i] = (i % 5) ? 1 : -1; }
        if (oracle_icm_pair(n, rp, col, xa, xb, 0x9E3779B9u, mask) < 0) bad = 1;
        free(rp); free(col); free(w);
    }
    uint64_t Wt[5] = {1ull << 32, 0, 12345, 1ull << 31, 7};
    int32_t nr[5];
    if (oracle_resample_counts(5, Wt, 0xDEADBEEFCAFEF00Dull, nr) == 0) bad = 1;
    if (!bad) printf("oracle sanitizer driver ok\n");
    return bad;
}
