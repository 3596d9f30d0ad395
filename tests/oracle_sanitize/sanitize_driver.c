/* Runs the FP64 oracle (compiled into this program with the address and
 * undefined-behaviour sanitizers) over every code path the pins use: D3Q19 and
 * D2Q9, one and two components, one and two n_s fields, reservoirs on each
 * axis, both forcing schemes, moments and single-cell updates, on domains
 * with extents 1 to 9.  Each case checks per-component mass conservation
 * where it must hold; any out-of-bounds access, use of uninitialised memory
 * the sanitizers see, or undefined arithmetic aborts the program. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "hmcsc_oracle.h"

static unsigned long long rng_state = 88172645463325252ULL;
static double urand(void)
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) / 9007199254740992.0;
}

static int run_case(int lattice, int nx, int ny, int nz, int ncomp, int c_ns, int n_res, int forcing, int steps)
{
    href_params p;
    memset(&p, 0, sizeof p);
    p.lattice = lattice;
    p.nx = nx; p.ny = ny; p.nz = nz;
    p.ncomp = ncomp; p.c_ns = c_ns; p.n_res = n_res; p.nthreads = 1;
    p.tau[0] = 0.8; p.tau[1] = 1.2;
    p.G = ncomp == 2 ? 0.7 : 0.0;
    p.G_ads[0] = 0.2; p.G_ads[1] = -0.15;
    p.F_ext[0] = 2e-4; p.F_ext[1] = -1e-4; p.F_ext[2] = lattice == 19 ? 3e-4 : 0.0;
    p.g_scale = 1.0;
    p.forcing = forcing;
    const int dims[3] = {nx, ny, nz};
    for (int r = 0; r < n_res; ++r) {
        p.res[r].axis = r % (lattice == 19 ? 3 : 2);
        p.res[r].lo = 0;
        p.res[r].hi = dims[p.res[r].axis] > 1 ? 1 : 0;
        p.res[r].rho[0] = 0.6; p.res[r].rho[1] = 0.4;
    }
    const int q = lattice;
    const long N = (long)nx * ny * nz;
    double* ns = malloc(sizeof(double) * c_ns * N);
    double* rho = malloc(sizeof(double) * ncomp * N);
    double* f = malloc(sizeof(double) * ncomp * q * N);
    double* work = malloc(sizeof(double) * ncomp * q * N);
    double* rf = malloc(sizeof(double) * ncomp * N);
    double* u = malloc(sizeof(double) * 3 * N);
    double* pr = malloc(sizeof(double) * N);
    double* ft = malloc(sizeof(double) * ncomp * 3 * N);
    const double choices[5] = {0.0, 0.05, 0.4, 0.9, 1.0};
    for (long k = 0; k < c_ns * N; ++k) ns[k] = choices[(int)(urand() * 5) % 5];
    for (long k = 0; k < ncomp * N; ++k) rho[k] = 0.3 + 0.4 * urand();
    if (href_init(&p, rho, f)) return 1;
    double m0[2] = {0, 0};
    for (int s = 0; s < ncomp; ++s)
        for (long k = 0; k < q * N; ++k) m0[s] += f[(long)s * q * N + k];
    if (href_run(&p, ns, f, work, steps)) return 2;
    if (href_moments(&p, ns, f, rf, u, pr, ft)) return 3;
    long cells[3] = {0, N / 2, N - 1};
    double* out = malloc(sizeof(double) * ncomp * q * 3);
    if (href_cell_update(&p, ns, f, 3, cells, out)) return 4;
    for (long k = 0; k < ncomp * q * N; ++k)
        if (!isfinite(f[k])) return 5;
    if (n_res == 0) {
        for (int s = 0; s < ncomp; ++s) {
            double m = 0;
            for (long k = 0; k < q * N; ++k) m += f[(long)s * q * N + k];
            if (fabs(m - m0[s]) > 1e-11 * m0[s]) return 6;
        }
    }
    free(ns); free(rho); free(f); free(work); free(rf); free(u); free(pr); free(ft); free(out);
    return 0;
}

int main(void)
{
    const int shapes[][3] = {{1, 1, 1}, {3, 1, 2}, {5, 4, 3}, {9, 2, 7}, {2, 7, 5}};
    int n = 0;
    for (int sh = 0; sh < 5; ++sh)
        for (int ncomp = 1; ncomp <= 2; ++ncomp)
            for (int c_ns = 1; c_ns <= ncomp; ++c_ns)
                for (int forcing = 0; forcing <= 1; ++forcing)
                    for (int n_res = 0; n_res <= 3; n_res += 3) {
                        const int* d = shapes[sh];
                        int rc = run_case(19, d[0], d[1], d[2], ncomp, c_ns, n_res, forcing, 6);
                        if (rc) { printf("D3Q19 case %d failed: %d\n", n, rc); return 1; }
                        rc = run_case(9, d[0], d[1], 1, ncomp, c_ns, n_res > 0 ? 2 : 0, forcing, 6);
                        if (rc) { printf("D2Q9 case %d failed: %d\n", n, rc); return 1; }
                        ++n;
                    }
    printf("sanitized oracle: %d cases passed\n", 2 * n);
    return 0;
}
