/* A plain C program that drives the library through include/lbm.h only: no
 * Python, no PyTorch, library-owned device memory on the default stream.
 *
 * Two-component droplet (Sec. 3.3 set-up) in a ragged 24 x 20 x 18 periodic
 * box with a gray medium, solid voxels and adhesion, FP64 storage:
 *   1. invalid parameters are rejected with LBM_EINVAL and no context;
 *   2. 200 steps conserve each component's mass (Eq. rho_BGK sums) to 1e-12;
 *   3. a checkpoint taken with lbm_get_populations and restored with
 *      lbm_set_populations / lbm_set_time continues bit for bit like the
 *      uninterrupted run (FP64 totals and densities after 50 more steps);
 *   4. a server (shortest-first sharing, two slots) serves three requests of
 *      the same problem with different step budgets; each result's densities
 *      and totals equal those of a context stepped alone as far.
 * Prints "C ABI OK" and exits 0 on success, 1 otherwise. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "lbm.h"

#define NX 24
#define NY 20
#define NZ 18
#define N (NX * NY * NZ)

static int fail(const char* what, int rc)
{
    printf("FAIL %s: %d (%s)\n", what, rc, lbm_strerror(rc));
    return 1;
}

int main(void)
{
    static float ns[N];
    static double rho[2 * N];
    const double c[3] = {(NX - 1) / 2.0, (NY - 1) / 2.0, (NZ - 1) / 2.0};
    for (int z = 0; z < NZ; ++z)
        for (int y = 0; y < NY; ++y)
            for (int x = 0; x < NX; ++x) {
                const int n = (z * NY + y) * NX + x;
                const double dx = x - c[0], dy = y - c[1], dz = z - c[2];
                const int in = dx * dx + dy * dy + dz * dz <= 36.0;
                rho[n] = in ? 1.0 : 0.03;
                rho[N + n] = in ? 0.03 : 1.0;
                ns[n] = (x == 0 && y < 4) ? 1.0f : 0.1f;
            }

    lbm_params p;
    memset(&p, 0, sizeof(p));
    p.ncomp = 2;
    p.c_ns = 1;
    p.tau[0] = p.tau[1] = 1.0;
    p.G_inter = 0.9;
    p.G_ads[0] = 0.1;
    p.G_ads[1] = -0.1;
    p.g_scale = 3.0;
    p.storage = LBM_F64;
    p.forcing = LBM_FORCING_SHAN_CHEN;
    const lbm_domain d = {NX, NY, NZ};

    lbm_ctx* ctx = NULL;
    lbm_params bad = p;
    bad.tau[0] = 0.4;
    int rc = lbm_create(&d, ns, rho, &bad, NULL, NULL, &ctx);
    if (rc != LBM_EINVAL || ctx != NULL) return fail("tau <= 1/2 accepted", rc);

    rc = lbm_create(&d, ns, rho, &p, NULL, NULL, &ctx);
    if (rc != LBM_OK) return fail("lbm_create", rc);
    lbm_totals t0, t1, ta, tb;
    if ((rc = lbm_totals_get(ctx, &t0)) != LBM_OK) return fail("lbm_totals_get", rc);
    if ((rc = lbm_step(ctx, 200)) != LBM_OK) return fail("lbm_step", rc);
    if ((rc = lbm_totals_get(ctx, &t1)) != LBM_OK) return fail("lbm_totals_get", rc);
    for (int s = 0; s < 2; ++s)
        if (!t1.finite || fabs(t1.mass[s] / t0.mass[s] - 1.0) > 1e-12) {
            printf("FAIL mass %d: %.17g -> %.17g\n", s, t0.mass[s], t1.mass[s]);
            return 1;
        }
    if (t1.time != 200) return fail("time after 200 steps", (int)t1.time);

    double* f = malloc(sizeof(double) * 2 * 19 * N);
    double* ra = malloc(sizeof(double) * 2 * N);
    double* rb = malloc(sizeof(double) * 2 * N);
    if (!f || !ra || !rb) return fail("malloc", 0);
    if ((rc = lbm_get_populations(ctx, f)) != LBM_OK) return fail("lbm_get_populations", rc);
    if ((rc = lbm_step(ctx, 50)) != LBM_OK) return fail("lbm_step", rc);
    if ((rc = lbm_moments(ctx, ra, NULL, NULL, &ta)) != LBM_OK) return fail("lbm_moments", rc);
    if ((rc = lbm_set_populations(ctx, f)) != LBM_OK) return fail("lbm_set_populations", rc);
    if ((rc = lbm_set_time(ctx, 200)) != LBM_OK) return fail("lbm_set_time", rc);
    if ((rc = lbm_step(ctx, 50)) != LBM_OK) return fail("lbm_step", rc);
    if ((rc = lbm_moments(ctx, rb, NULL, NULL, &tb)) != LBM_OK) return fail("lbm_moments", rc);
    if (memcmp(ra, rb, sizeof(double) * 2 * N) != 0 || memcmp(ta.mass, tb.mass, sizeof(ta.mass)) != 0 ||
        memcmp(ta.momentum, tb.momentum, sizeof(ta.momentum)) != 0 || ta.time != 250 || tb.time != 250)
        return fail("checkpoint restart differs", 0);
    free(f);
    lbm_destroy(ctx);

    lbm_server_cfg cfg;
    memset(&cfg, 0, sizeof(cfg));
    cfg.max_slots = 2;
    cfg.steps_per_tick = 16;
    cfg.storage = LBM_F64;
    cfg.ncomp = 2;
    cfg.c_ns = 1;
    cfg.max_cells = N;
    cfg.policy = LBM_SERVE_SHORTEST_FIRST;
    lbm_server* srv = NULL;
    if ((rc = lbm_server_create(&cfg, NULL, &srv)) != LBM_OK) return fail("lbm_server_create", rc);
    const int64_t budget[3] = {70, 16, 33};
    uint64_t ticket[3];
    double* out[3];
    for (int k = 0; k < 3; ++k) {
        out[k] = malloc(sizeof(double) * 2 * N);
        if (!out[k]) return fail("malloc", 0);
        lbm_request rq;
        memset(&rq, 0, sizeof(rq));
        rq.dom = d;
        rq.n_s = ns;
        rq.rho_init = rho;
        rq.params = p;
        rq.max_steps = budget[k];
        rq.rho_out = out[k];
        if ((rc = lbm_batch_submit(srv, &rq, &ticket[k])) != LBM_OK) return fail("lbm_batch_submit", rc);
    }
    for (int k = 0; k < 3; ++k) {
        lbm_result res;
        if ((rc = lbm_batch_wait(srv, ticket[k], 60.0, &res)) != LBM_OK) return fail("lbm_batch_wait", rc);
        if (res.status != LBM_OK || res.steps_done != budget[k]) return fail("request status", res.status);
        lbm_ctx* alone = NULL;
        if ((rc = lbm_create(&d, ns, rho, &p, NULL, NULL, &alone)) != LBM_OK) return fail("lbm_create", rc);
        if ((rc = lbm_step(alone, budget[k])) != LBM_OK) return fail("lbm_step", rc);
        if ((rc = lbm_moments(alone, ra, NULL, NULL, &ta)) != LBM_OK) return fail("lbm_moments", rc);
        lbm_destroy(alone);
        if (memcmp(ra, out[k], sizeof(double) * 2 * N) != 0 ||
            memcmp(ta.mass, res.totals.mass, sizeof(ta.mass)) != 0 ||
            memcmp(ta.momentum, res.totals.momentum, sizeof(ta.momentum)) != 0)
            return fail("served result differs from the context stepped alone", k);
        free(out[k]);
    }
    lbm_server_destroy(srv);
    free(ra);
    free(rb);
    printf("mass %.17g %.17g  momentum %.3e %.3e %.3e\nC ABI OK\n", t1.mass[0], t1.mass[1], t1.momentum[0],
           t1.momentum[1], t1.momentum[2]);
    return 0;
}
