/*
 * Plain FP64 CPU oracle of the HMCSC lattice Boltzmann update.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark to check the GPU library, never by it.
 *
 * It follows the paper step by step, in its notation, with push streaming as
 * Eq. (LGS) is written:
 *   1. zeroth and first moments of every cell         Eqs. (rho_BGK), (mom_BGK)
 *   2. common velocity u' of the components           Eq. (SC_u_eq), first term
 *   3. cohesion, adhesion and external forces         Eqs. (SC_F_inter), (SC_F_ads), (SC_F_ext)
 *   4. force-shifted equilibrium velocity             Eq. (SC_u_eq)
 *   5. equilibrium, BGK relaxation and partial bounce-back with the
 *      pre-collision populations, streamed to x + c_i  Eqs. (Maxwell), (LGS)
 *   6. density reservoirs: reset to the rest equilibrium of the prescribed
 *      densities (Sec. 4 and Sec. 3.4 prescribe densities there; the mechanism
 *      is not stated, this is the reading taken).
 * Macroscopic outputs: u_macro of Eq. (HMCSC_u_macro) and p of Eq. (SC_pressure).
 *
 * The alternative the paper contrasts with (Appendix, Guo vs. Shan-Chen
 * forcing), forcing = HREF_FORCING_GUO: the grayscale scheme GS-WBS of
 * Eq. (GS-WBS).  Steps 1 and 3 are the same; the equilibrium of every
 * component is taken at u_macro of Eq. (HMCSC_u_macro) instead of step 4's
 * velocity, and (1 - n_s) times the forcing term of Guo et al. (2002),
 * evaluated with F_tot,sigma and u_macro, is added to the post-collision value.
 *
 * Readings of the paper taken here (the paper is silent or ambiguous):
 *   - The interaction stencils of Eqs. (SC_F_inter), (SC_F_ads) weight the
 *     neighbours with g_scale*w_i.  g_scale = 1 is the literal text; g_scale = 3
 *     (= 1/c_s^2) is the normalisation under which the paper's G_inter = 1.75
 *     separates the phases at all (Table 1, Sec. 3.3).  The pressure of
 *     Eq. (SC_pressure) uses the same factor so it stays the mechanical pressure.
 *   - u_sigma in Eq. (SC_u_eq) is the raw first moment of Eq. (mom_BGK), not
 *     weighted by (1 - n_s).
 *   - Densities entering the forces are those of every cell, solid or not
 *     (every cell holds every component, Sec. 2).
 *   - rho_sigma = 0: the component is absent, its equilibrium is zero and no
 *     force shift is applied.
 *
 * Parity pins (closed forms, invariants, printed values) live in tests/.
 */
#include "hmcsc_oracle.h"

#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXQ 19

/* D3Q19 velocity set in the order printed in Appendix A (Velocity Sets). */
static const int32_t D3Q19_C[19][3] = {
    {0, 0, 0},   {-1, 0, 0}, {0, -1, 0}, {0, 0, -1}, {-1, -1, 0},
    {-1, 1, 0},  {-1, 0, -1}, {-1, 0, 1}, {0, -1, -1}, {0, -1, 1},
    {1, 0, 0},   {0, 1, 0},  {0, 0, 1},  {1, 1, 0},  {1, -1, 0},
    {1, 0, 1},   {1, 0, -1}, {0, 1, 1},  {0, 1, -1}};

/* D2Q9 velocity set in the order printed in Appendix A (Velocity Sets). */
static const int32_t D2Q9_C[9][3] = {
    {0, 0, 0},  {-1, 1, 0}, {-1, 0, 0}, {-1, -1, 0}, {0, -1, 0},
    {1, -1, 0}, {1, 0, 0},  {1, 1, 0},  {0, 1, 0}};

static const double CS2 = 1.0 / 3.0; /* lattice speed of sound squared, both sets */

typedef struct {
    int q;
    int c[MAXQ][3];
    double w[MAXQ];
    int opp[MAXQ];
} lattice_t;

/* Weights by |c|^2 as stated with the velocity sets in Appendix A. */
static int make_lattice(int32_t which, lattice_t* L)
{
    const int32_t(*c)[3];
    double w0, w1, w2;
    if (which == 19) {
        L->q = 19; c = D3Q19_C; w0 = 1.0 / 3.0; w1 = 1.0 / 18.0; w2 = 1.0 / 36.0;
    } else if (which == 9) {
        L->q = 9; c = D2Q9_C; w0 = 4.0 / 9.0; w1 = 1.0 / 9.0; w2 = 1.0 / 36.0;
    } else {
        return -1;
    }
    for (int i = 0; i < L->q; ++i) {
        int len2 = 0;
        for (int a = 0; a < 3; ++a) {
            L->c[i][a] = c[i][a];
            len2 += c[i][a] * c[i][a];
        }
        L->w[i] = len2 == 0 ? w0 : (len2 == 1 ? w1 : w2);
    }
    /* opposite direction: the one with c_j = -c_i (i = 0 is its own opposite) */
    for (int i = 0; i < L->q; ++i) {
        L->opp[i] = -1;
        for (int j = 0; j < L->q; ++j)
            if (c[j][0] == -c[i][0] && c[j][1] == -c[i][1] && c[j][2] == -c[i][2])
                L->opp[i] = j;
        if (L->opp[i] < 0) return -1;
    }
    return 0;
}

int href_lattice(int32_t which, int32_t* q, int32_t* c, double* w, int32_t* opp)
{
    lattice_t L;
    if (make_lattice(which, &L)) return -1;
    *q = L.q;
    for (int i = 0; i < L.q; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
        w[i] = L.w[i];
        opp[i] = L.opp[i];
    }
    return 0;
}

static int check_params(const href_params* p, lattice_t* L)
{
    if (make_lattice(p->lattice, L)) return -1;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
    if (p->lattice == 9 && p->nz != 1) return -1;
    if (p->ncomp < 1 || p->ncomp > 2) return -1;
    if (p->c_ns < 1 || p->c_ns > 2 || p->c_ns > p->ncomp) return -1;
    if (p->n_res < 0 || p->n_res > HREF_MAX_RES) return -1;
    for (int s = 0; s < p->ncomp; ++s)
        if (!(p->tau[s] > 0.5)) return -1;
    if (p->forcing != HREF_FORCING_SHAN_CHEN && p->forcing != HREF_FORCING_GUO) return -1;
    for (int r = 0; r < p->n_res; ++r) {
        const href_reservoir* R = &p->res[r];
        if (R->axis < 0 || R->axis > 2 || R->lo < 0 || R->hi < R->lo) return -1;
    }
    return 0;
}

static int64_t ncells(const href_params* p) { return (int64_t)p->nx * p->ny * p->nz; }

static int64_t cell_of(const href_params* p, int x, int y, int z)
{
    return ((int64_t)z * p->ny + y) * p->nx + x;
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

static double ns_at(const href_params* p, const double* ns, int s, int64_t n)
{
    return ns[(p->c_ns == 2 ? s : 0) * ncells(p) + n];
}

/* Eq. (rho_BGK) for one cell and component. */
static double density_at(const href_params* p, const lattice_t* L, const double* f, int s, int64_t n)
{
    double r = 0.0;
    for (int i = 0; i < L->q; ++i) r += f[(s * L->q + i) * ncells(p) + n];
    return r;
}

/* Index of the reservoir containing the cell, or -1. */
static int reservoir_of(const href_params* p, int x, int y, int z)
{
    const int xyz[3] = {x, y, z};
    for (int r = 0; r < p->n_res; ++r)
        if (xyz[p->res[r].axis] >= p->res[r].lo && xyz[p->res[r].axis] < p->res[r].hi) return r;
    return -1;
}

/*
 * Forcing term of Guo, Zheng and Shi (Phys. Rev. E 65, 046308, 2002), which
 * the GS-WBS of Eq. (GS-WBS) uses, for direction i, force F and velocity u:
 *   F_i = (1 - 1/(2 tau)) w_i [ (c_i - u).F / c_s^2 + (c_i.u)(c_i.F) / c_s^4 ].
 */
static double guo_term(const lattice_t* L, int i, double tau, const double u[3], const double F[3])
{
    double cF = 0.0, uF = 0.0, cu = 0.0;
    for (int a = 0; a < 3; ++a) {
        cF += L->c[i][a] * F[a];
        uF += u[a] * F[a];
        cu += L->c[i][a] * u[a];
    }
    return (1.0 - 1.0 / (2.0 * tau)) * L->w[i] * ((cF - uF) / CS2 + cu * cF / (CS2 * CS2));
}

/*
 * Local collision at cell (x,y,z): post[s][i] is the right-hand side of
 * Eq. (LGS) (or of Eq. (GS-WBS) with Guo forcing), i.e. what leaves the cell
 * in direction i.  The densities of the
 * neighbours come from rho_field when given, otherwise they are summed from f.
 * ftot (optional) receives F_tot,sigma.
 */
static void collide_at(const href_params* p, const lattice_t* L, const double* ns,
                       const double* f, const double* rho_field, int x, int y, int z,
                       double post[2][MAXQ], double ftot[2][3], double ueq_out[2][3])
{
    const int Q = L->q;
    const int64_t N = ncells(p);
    const int64_t n = cell_of(p, x, y, z);
    double fl[2][MAXQ], rho_s[2] = {0.0, 0.0}, j[2][3] = {{0.0}};

    /* 1. Eqs. (rho_BGK), (mom_BGK): rho_sigma and rho_sigma u_sigma */
    for (int s = 0; s < p->ncomp; ++s) {
        for (int i = 0; i < Q; ++i) fl[s][i] = f[(s * Q + i) * N + n];
        for (int i = 0; i < Q; ++i) {
            rho_s[s] += fl[s][i];
            for (int a = 0; a < 3; ++a) j[s][a] += fl[s][i] * L->c[i][a];
        }
    }
    double rho = 0.0;
    for (int s = 0; s < p->ncomp; ++s) rho += rho_s[s];

    /* 2. common velocity, first term of Eq. (SC_u_eq) */
    double num[3] = {0.0, 0.0, 0.0}, den = 0.0, up[3];
    for (int s = 0; s < p->ncomp; ++s) {
        for (int a = 0; a < 3; ++a) num[a] += j[s][a] / p->tau[s];
        den += rho_s[s] / p->tau[s];
    }
    for (int a = 0; a < 3; ++a) up[a] = den > 0.0 ? num[a] / den : 0.0;

    /* 3. total force per component */
    double Ft[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int s = 0; s < p->ncomp; ++s) {
        double Finter[3] = {0.0, 0.0, 0.0}, Fads[3] = {0.0, 0.0, 0.0}, Fext[3];

        /* 3a. Eq. (SC_F_inter): -rho_s G sum_i W_i rho_sbar(x + c_i) c_i */
        if (p->ncomp == 2) {
            const int sb = 1 - s;
            double g[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < Q; ++i) {
                const int64_t nb = cell_of(p, wrap(x + L->c[i][0], p->nx), wrap(y + L->c[i][1], p->ny),
                                           wrap(z + L->c[i][2], p->nz));
                const double r_nb = rho_field ? rho_field[sb * N + nb] : density_at(p, L, f, sb, nb);
                for (int a = 0; a < 3; ++a) g[a] += p->g_scale * L->w[i] * r_nb * L->c[i][a];
            }
            for (int a = 0; a < 3; ++a) Finter[a] = -rho_s[s] * p->G * g[a];
        }
        /* 3b. Eq. (SC_F_ads) with s = n_s,sigma */
        {
            double g[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < Q; ++i) {
                const int64_t nb = cell_of(p, wrap(x + L->c[i][0], p->nx), wrap(y + L->c[i][1], p->ny),
                                           wrap(z + L->c[i][2], p->nz));
                const double s_nb = ns_at(p, ns, s, nb);
                for (int a = 0; a < 3; ++a) g[a] += p->g_scale * L->w[i] * s_nb * L->c[i][a];
            }
            for (int a = 0; a < 3; ++a) Fads[a] = -rho_s[s] * p->G_ads[s] * g[a];
        }
        /* 3c. Eq. (SC_F_ext) */
        for (int a = 0; a < 3; ++a) Fext[a] = rho > 0.0 ? rho_s[s] / rho * p->F_ext[a] : 0.0;

        for (int a = 0; a < 3; ++a) Ft[s][a] = Finter[a] + Fads[a] + Fext[a];
        if (ftot)
            for (int a = 0; a < 3; ++a) ftot[s][a] = Ft[s][a];
    }

    /* 4. velocity of the equilibrium: Eq. (SC_u_eq) for the HMCSC; for the
     * GS-WBS with Guo forcing the macroscopic velocity of Eq. (HMCSC_u_macro),
     * common to both components */
    double um[3] = {0.0, 0.0, 0.0};
    if (p->forcing == HREF_FORCING_GUO)
        for (int a = 0; a < 3; ++a) {
            double m = 0.0;
            for (int s = 0; s < p->ncomp; ++s)
                m += (1.0 - ns_at(p, ns, s, n)) * (j[s][a] + 0.5 * Ft[s][a]);
            um[a] = rho > 0.0 ? m / rho : 0.0;
        }

    for (int s = 0; s < p->ncomp; ++s) {
        const double nsx = ns_at(p, ns, s, n);
        double ueq[3];
        for (int a = 0; a < 3; ++a)
            ueq[a] = p->forcing == HREF_FORCING_GUO
                         ? um[a]
                         : up[a] + (rho_s[s] > 0.0 ? p->tau[s] * Ft[s][a] / rho_s[s] : 0.0);
        if (ueq_out)
            for (int a = 0; a < 3; ++a) ueq_out[s][a] = ueq[a];

        /* 5. Eq. (Maxwell) and Eq. (LGS), or Eq. (GS-WBS) with the Guo term */
        const double uu = ueq[0] * ueq[0] + ueq[1] * ueq[1] + ueq[2] * ueq[2];
        for (int i = 0; i < Q; ++i) {
            const double cu = L->c[i][0] * ueq[0] + L->c[i][1] * ueq[1] + L->c[i][2] * ueq[2];
            const double feq = L->w[i] * rho_s[s] *
                               (1.0 + cu / CS2 + (cu * cu) / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
            post[s][i] = (1.0 - nsx) * fl[s][i] - (1.0 - nsx) / p->tau[s] * (fl[s][i] - feq) +
                         nsx * fl[s][L->opp[i]];
            if (p->forcing == HREF_FORCING_GUO)
                post[s][i] += (1.0 - nsx) * guo_term(L, i, p->tau[s], ueq, Ft[s]);
        }
    }
}

/* Rest equilibrium w_i rho of Eq. (Maxwell) with u = 0. */
static void reset_reservoirs(const href_params* p, const lattice_t* L, double* f)
{
    const int64_t N = ncells(p);
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const int r = reservoir_of(p, x, y, z);
                if (r < 0) continue;
                const int64_t n = cell_of(p, x, y, z);
                for (int s = 0; s < p->ncomp; ++s)
                    for (int i = 0; i < L->q; ++i) f[(s * L->q + i) * N + n] = L->w[i] * p->res[r].rho[s];
            }
}

static int nthreads_of(const href_params* p)
{
#ifdef _OPENMP
    return p->nthreads > 0 ? p->nthreads : omp_get_max_threads();
#else
    (void)p;
    return 1;
#endif
}

int href_init(const href_params* p, const double* rho_init, double* f)
{
    lattice_t L;
    if (check_params(p, &L)) return -1;
    const int64_t N = ncells(p);
    for (int s = 0; s < p->ncomp; ++s)
        for (int i = 0; i < L.q; ++i)
            for (int64_t n = 0; n < N; ++n) f[(s * L.q + i) * N + n] = L.w[i] * rho_init[s * N + n];
    reset_reservoirs(p, &L, f);
    return 0;
}

static void density_field(const href_params* p, const lattice_t* L, const double* f, double* rho, int nt)
{
    const int64_t N = ncells(p);
    (void)nt;
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t n = 0; n < N; ++n)
        for (int s = 0; s < p->ncomp; ++s) rho[s * N + n] = density_at(p, L, f, s, n);
}

static int step_with(const href_params* p, const lattice_t* L, const double* ns, const double* f_in,
                     double* f_out, double* rho)
{
    const int64_t N = ncells(p);
    const int nt = nthreads_of(p);
    (void)nt;
    density_field(p, L, f_in, rho, nt);
    const int rows = p->ny * p->nz;
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int zy = 0; zy < rows; ++zy) {
        const int z = zy / p->ny, y = zy % p->ny;
        double post[2][MAXQ];
        for (int x = 0; x < p->nx; ++x) {
            collide_at(p, L, ns, f_in, rho, x, y, z, post, NULL, NULL);
            /* push streaming: f_i(x + c_i, t + 1) = post_i(x) */
            for (int s = 0; s < p->ncomp; ++s)
                for (int i = 0; i < L->q; ++i) {
                    const int64_t dst = cell_of(p, wrap(x + L->c[i][0], p->nx), wrap(y + L->c[i][1], p->ny),
                                                wrap(z + L->c[i][2], p->nz));
                    f_out[(s * L->q + i) * N + dst] = post[s][i];
                }
        }
    }
    reset_reservoirs(p, L, f_out);
    return 0;
}

int href_step(const href_params* p, const double* ns, const double* f_in, double* f_out)
{
    lattice_t L;
    if (check_params(p, &L)) return -1;
    double* rho = (double*)malloc(sizeof(double) * (size_t)(p->ncomp * ncells(p)));
    if (!rho) return -2;
    step_with(p, &L, ns, f_in, f_out, rho);
    free(rho);
    return 0;
}

int href_run(const href_params* p, const double* ns, double* f, double* work, int64_t nsteps)
{
    lattice_t L;
    if (check_params(p, &L)) return -1;
    if (nsteps < 0) return -1;
    const int64_t total = (int64_t)p->ncomp * L.q * ncells(p);
    double* rho = (double*)malloc(sizeof(double) * (size_t)(p->ncomp * ncells(p)));
    if (!rho) return -2;
    double* a = f;
    double* b = work;
    for (int64_t t = 0; t < nsteps; ++t) {
        step_with(p, &L, ns, a, b, rho);
        double* tmp = a; a = b; b = tmp;
    }
    if (a != f) memcpy(f, a, sizeof(double) * (size_t)total);
    free(rho);
    return 0;
}

int href_moments(const href_params* p, const double* ns, const double* f, double* rho, double* u,
                 double* pr, double* ftot)
{
    lattice_t L;
    if (check_params(p, &L)) return -1;
    const int64_t N = ncells(p);
    double* rf = (double*)malloc(sizeof(double) * (size_t)(p->ncomp * N));
    if (!rf) return -2;
    const int nt = nthreads_of(p);
    density_field(p, &L, f, rf, nt);
    const int rows = p->ny * p->nz;
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int zy = 0; zy < rows; ++zy) {
        const int z = zy / p->ny, y = zy % p->ny;
        double post[2][MAXQ], Ft[2][3];
        for (int x = 0; x < p->nx; ++x) {
            const int64_t n = cell_of(p, x, y, z);
            collide_at(p, &L, ns, f, rf, x, y, z, post, Ft, NULL);
            double rho_tot = 0.0;
            for (int s = 0; s < p->ncomp; ++s) rho_tot += rf[s * N + n];
            if (rho)
                for (int s = 0; s < p->ncomp; ++s) rho[s * N + n] = rf[s * N + n];
            if (ftot)
                for (int s = 0; s < p->ncomp; ++s)
                    for (int a = 0; a < 3; ++a) ftot[(s * 3 + a) * N + n] = Ft[s][a];
            if (u) {
                /* Eq. (HMCSC_u_macro) */
                for (int a = 0; a < 3; ++a) {
                    double m = 0.0;
                    for (int s = 0; s < p->ncomp; ++s) {
                        double js = 0.0;
                        for (int i = 0; i < L.q; ++i) js += f[(s * L.q + i) * N + n] * L.c[i][a];
                        m += (1.0 - ns_at(p, ns, s, n)) * (js + Ft[s][a] / 2.0);
                    }
                    u[a * N + n] = rho_tot > 0.0 ? m / rho_tot : 0.0;
                }
            }
            if (pr) {
                /* Eq. (SC_pressure), interaction term scaled like the force stencil */
                double inter = p->ncomp == 2 ? p->g_scale * p->G * rf[n] * rf[N + n] : 0.0;
                pr[n] = CS2 * (rho_tot + inter);
            }
        }
    }
    free(rf);
    return 0;
}

int href_cell_update(const href_params* p, const double* ns, const double* f_in, int64_t nc,
                     const int64_t* cells, double* out)
{
    lattice_t L;
    if (check_params(p, &L)) return -1;
    const int64_t N = ncells(p);
    const int Q = L.q;
    const int nt = nthreads_of(p);
    (void)nt;
    int bad = 0;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 16) reduction(| : bad)
    for (int64_t k = 0; k < nc; ++k) {
        const int64_t n = cells[k];
        if (n < 0 || n >= N) { bad = 1; continue; }
        const int x = (int)(n % p->nx), y = (int)((n / p->nx) % p->ny), z = (int)(n / ((int64_t)p->nx * p->ny));
        const int r = reservoir_of(p, x, y, z);
        double post[2][MAXQ];
        for (int i = 0; i < Q; ++i) {
            /* f_i(x, t + 1) left cell x - c_i in direction i */
            collide_at(p, &L, ns, f_in, NULL, wrap(x - L.c[i][0], p->nx), wrap(y - L.c[i][1], p->ny),
                       wrap(z - L.c[i][2], p->nz), post, NULL, NULL);
            for (int s = 0; s < p->ncomp; ++s)
                out[(k * p->ncomp + s) * Q + i] = r >= 0 ? L.w[i] * p->res[r].rho[s] : post[s][i];
        }
    }
    return bad ? -1 : 0;
}
