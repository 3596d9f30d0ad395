/*
 * Plain FP64 CPU oracle of the homogenized multi-component Shan-Chen lattice
 * Boltzmann method (HMCSC): grayscale partial bounce-back (Walsh-Burwinkle-Saar)
 * combined with the multi-component Shan-Chen model and its forcing scheme.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.  It is
 * loaded by the test-suite, by the smoke check and by the CPU-baseline leg of the
 * benchmark, never by the product path.  It shares no source, header, table or
 * helper with the GPU library.
 *
 * Array layouts (all host memory, caller-owned, x fastest):
 *   cell index        n = (z*ny + y)*nx + x,  N = nx*ny*nz
 *   populations f     f[(s*Q + i)*N + n]      s = component, i = direction
 *   bounce-back frac. ns[k*N + n]             k = 0 (shared) or k = s (c_ns == 2)
 *   densities         rho[s*N + n]
 *   velocity          u[a*N + n]              a = 0,1,2 (x,y,z)
 *   total force       ftot[(s*3 + a)*N + n]
 * The populations are the pre-collision state f(x,t) of Eq. (LGS).
 */
#ifndef HMCSC_ORACLE_H
#define HMCSC_ORACLE_H

#include <stdint.h>

#define HREF_MAX_RES 4

/* A slab of cells whose pre-collision state is reset to the rest equilibrium
 * of the prescribed densities after every streaming step (density reservoir). */
typedef struct {
    int32_t axis; /* 0: x, 1: y, 2: z */
    int32_t lo;   /* first coordinate inside the slab            */
    int32_t hi;   /* one past the last coordinate inside the slab */
    int32_t pad;
    double rho[2];
} href_reservoir;

typedef struct {
    int32_t lattice;  /* 19: D3Q19, 9: D2Q9 (2-D, requires nz == 1)     */
    int32_t nx, ny, nz;
    int32_t ncomp;    /* number of fluid components, 1 or 2            */
    int32_t c_ns;     /* number of bounce-back-fraction fields, 1 or 2 */
    int32_t n_res;    /* number of reservoirs, 0..HREF_MAX_RES         */
    int32_t nthreads; /* OpenMP threads; 0 = runtime default           */
    double tau[2];    /* relaxation time per component                 */
    double G;         /* fluid-fluid interaction G_inter,12 = G_inter,21 */
    double G_ads[2];  /* fluid-solid interaction per component          */
    double F_ext[3];  /* external body force density                    */
    double g_scale;   /* interaction stencils weight neighbours by g_scale*w_i */
    href_reservoir res[HREF_MAX_RES];
    int32_t forcing;  /* HREF_FORCING_SHAN_CHEN: the HMCSC, Eq. (HMCSC)           */
                      /* HREF_FORCING_GUO: the GS-WBS with Guo forcing, Eq. (GS-WBS) */
    int32_t pad;
} href_params;

#define HREF_FORCING_SHAN_CHEN 0
#define HREF_FORCING_GUO 1

/* Velocity set: q directions, c[3*i + a], weights w[i], opposite opp[i]. */
int href_lattice(int32_t lattice, int32_t* q, int32_t* c, double* w, int32_t* opp);

/* f = rest equilibrium of rho_init (reservoir slabs: of their densities). */
int href_init(const href_params* p, const double* rho_init, double* f);

/* One time step: f_out = state at t+1 from the state f_in at t. */
int href_step(const href_params* p, const double* ns, const double* f_in, double* f_out);

/* nsteps time steps in place on f; work is a second buffer of the same size. */
int href_run(const href_params* p, const double* ns, double* f, double* work, int64_t nsteps);

/* Macroscopic fields of the state f (any output pointer may be NULL). */
int href_moments(const href_params* p, const double* ns, const double* f,
                 double* rho, double* u, double* pr, double* ftot);

/* The state at t+1 in a list of cells only: out[(k*ncomp + s)*Q + i]. */
int href_cell_update(const href_params* p, const double* ns, const double* f_in,
                     int64_t ncells, const int64_t* cells, double* out);

#endif
