/*
 * Drives the host-side paths of the C ABI (include/pa.h) that need no
 * device work -- graph validation, schedule checks and planning, table
 * building, checkpoint and batch refusals, the pool's admission logic -- so
 * that a build of the library's host code with AddressSanitizer and
 * UndefinedBehaviorSanitizer checks them. Test infrastructure
 * (tests/test_sanitizers.py builds and runs it on a machine without a GPU);
 * exits non-zero on an unexpected status, and the sanitizers abort on any
 * memory or undefined-behaviour error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pa.h"

static int bad = 0;

static void expect(pa_status got, pa_status want, const char *what)
{
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, pa_last_error());
        bad = 1;
    }
}

/* Ring with chords i -- i+5 (mod n); negative weights on odd index sums when signed. */
static void graph(int n, int sg, int32_t *rp, int32_t *col, int8_t *w)
{
    int e = 0;
    for (int i = 0; i < n; ++i) {
        rp[i] = e;
        int nb[4] = {(i + n - 5) % n, (i + n - 1) % n, (i + 1) % n, (i + 5) % n};
        for (int q = 0; q < 4; ++q) {
            int j = nb[q], lo = i < j ? i : j, hi = i < j ? j : i;
            col[e] = j;
            w[e] = (sg && ((lo + hi) & 1)) ? -1 : 1;
            ++e;
        }
    }
    rp[n] = e;
}

int main(void)
{
    enum { N = 64 };
    int32_t rp[N + 1], col[4 * N];
    int8_t w[4 * N];
    double beta[20];
    for (int k = 0; k < 20; ++k) beta[k] = 0.1 + 0.1 * k;
    pa_schedule sch;
    memset(&sch, 0, sizeof sch);
    sch.n_steps = 20;
    sch.beta = beta;
    sch.sweeps_per_step = 2;
    sch.as_stall_steps = 2;
    sch.as_max_level = 3;
    sch.as_frozen_inv = 8;
    sch.as_gamma = 0.8;
    sch.adapt_jump = 4;
    sch.adapt_num = 1;
    sch.adapt_den = 2;

    for (int sg = 0; sg < 2; ++sg) {
        graph(N, sg, rp, col, w);
        pa_solver *s = NULL;
        expect(pa_create(&s, N, rp, col, w), PA_OK, "pa_create");
        int64_t info[4];
        expect(pa_graph_info(s, info), PA_OK, "pa_graph_info");
        expect(pa_set_fault_step(s, 5), PA_OK, "pa_set_fault_step");
        expect(pa_set_fault_step(s, -2), PA_EINVAL, "fault step -2");
        expect(pa_set_fault_step(s, -1), PA_OK, "fault step off");
        size_t bytes = 0;
        for (int variant = 0; variant < 6; ++variant) {
            pa_schedule v = sch;
            v.as_enable = variant >= 1;
            v.nl_period = variant == 2 || variant == 3 ? 3 : 0;
            v.nl_kind = variant == 3;
            v.beta_adapt = variant == 4;
            v.sweep_kernel = variant == 5 ? 2 : 0;
            expect(pa_workspace_bytes(s, &v, 96, &bytes), PA_OK, "pa_workspace_bytes");
            size_t tb = 0;
            expect(pa_build_tables(&v, 4, 50, NULL, &tb), PA_OK, "pa_build_tables size");
            uint64_t *t = malloc(tb);
            expect(pa_build_tables(&v, 4, 50, t, &tb), PA_OK, "pa_build_tables");
            free(t);
        }
        /* refusals */
        pa_schedule b = sch;
        double dec[2] = {0.5, 0.4};
        b.beta = dec;
        b.n_steps = 2;
        expect(pa_workspace_bytes(s, &b, 32, &bytes), PA_EINVAL, "decreasing beta");
        b = sch;
        b.field_bits = 12;
        expect(pa_workspace_bytes(s, &b, 32, &bytes), PA_EINVAL, "field_bits 12");
        b.field_bits = 8;
        expect(pa_workspace_bytes(s, &b, 32, &bytes), PA_OK, "field_bits 8");
        b = sch;
        b.beta_adapt = 1;
        double geo[20];
        for (int k = 0; k < 20; ++k) geo[k] = 0.1 * (1 << (k / 4));
        b.beta = geo;
        expect(pa_workspace_bytes(s, &b, 32, &bytes), PA_EINVAL, "uneven grid");
        expect(pa_run(s, &sch, 32, 1, 0, NULL, 1 << 20, NULL), PA_EWORKSPACE, "null workspace");
        /* the static entry refuses what its workspace cannot hold, and
         * reports the missing device for the rest */
        for (int r = 1024; r <= 32768; r *= 32) {
            expect(pa_workspace_bytes(s, &sch, r, &bytes), PA_OK, "pa_workspace_bytes");
            expect(pa_run_static(s, &sch, r, 1, 0, NULL),
                   bytes > PA_STATIC_SCRATCH_BYTES ? PA_EWORKSPACE : PA_EDEVICE, "pa_run_static");
        }
        char blob[256];
        memset(blob, 0, sizeof blob);
        memcpy(blob, "PACKPT01", 8);
        expect(pa_checkpoint_load(s, &sch, 32, 1, 0, blob, sizeof blob, (void *)(uintptr_t)256, 1 << 20, NULL),
               PA_EINVAL, "bad checkpoint");
        /* fused batch plans and refusals (host only) */
        pa_fused_entry runs[2] = {{s, &sch, 40, 1, 0}, {s, &sch, 40, 2, 1}};
        pa_fused *f = NULL;
        expect(pa_fused_create(&f, runs, 2), PA_EINVAL, "solver twice");
        expect(pa_fused_create(&f, runs, 1), PA_OK, "pa_fused_create");
        size_t fb = 0;
        expect(pa_fused_workspace_bytes(f, &fb), PA_OK, "pa_fused_workspace_bytes");
        int64_t g[8 * 8];
        int32_t ng = 0;
        expect(pa_fused_info(f, g, 8, &ng), PA_OK, "pa_fused_info");
        expect(pa_fused_run(f, NULL, fb, NULL), PA_EWORKSPACE, "fused null workspace");
        expect(pa_fused_destroy(f), PA_OK, "pa_fused_destroy");
        /* pool admission (no device work before an advance) */
        pa_pool *p = NULL;
        expect(pa_pool_create(&p, (void *)(uintptr_t)(1 << 20), (size_t)64 << 20), PA_OK, "pa_pool_create");
        int64_t t1 = 0, t2 = 0;
        expect(pa_pool_submit(p, &runs[0], &t1), PA_OK, "pa_pool_submit");
        expect(pa_pool_submit(p, &runs[0], &t2), PA_EINVAL, "pool solver twice");
        expect(pa_pool_release(p, t1), PA_ESTATE, "release waiting");
        expect(pa_pool_cancel(p, t1), PA_OK, "pa_pool_cancel");
        int64_t pi[6];
        expect(pa_pool_info(p, pi), PA_OK, "pa_pool_info");
        expect(pa_pool_destroy(p), PA_OK, "pa_pool_destroy");
        expect(pa_destroy(s), PA_OK, "pa_destroy");
    }
    /* malformed graphs */
    graph(N, 0, rp, col, w);
    pa_solver *s = NULL;
    w[3] = 2;
    expect(pa_create(&s, N, rp, col, w), PA_EINVAL, "weight 2");
    w[3] = 1;
    col[0] = 0;
    expect(pa_create(&s, N, rp, col, w), PA_EINVAL, "self loop");
    expect(pa_create(&s, 1, rp, col, w), PA_ERANGE, "one node");
    if (!bad) printf("library host sanitizer driver ok\n");
    return bad;
}
