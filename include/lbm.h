/*
 * lbm.h - C ABI of the MI355X (gfx950) implementation of the homogenized
 * multi-component Shan-Chen lattice Boltzmann method (HMCSC): D3Q19, one or two
 * fluid components, grayscale partial bounce-back weighted by a per-voxel
 * bounce-back fraction n_s.
 *
 * One time step is Eq. (LGS) of Sec. 2 for every component sigma:
 *   f_i(x + c_i, t + 1) = (1 - n_s)(f_i - (f_i - f_i^eq)/tau_sigma) + n_s f_ibar(x, t)
 * with f^eq of Eq. (Maxwell) at the force-shifted velocity of Eq. (SC_u_eq), the
 * forces of Eqs. (SC_F_inter), (SC_F_ads), (SC_F_ext), the D3Q19 velocity set of
 * Appendix A, periodic streaming in x, y and z.  The bounce-back term uses the
 * pre-collision populations of the same cell (Appendix A, Eq. LBGKWBS).
 *
 * Conventions shared by every call:
 *   - Cells are indexed n = (z*ny + y)*nx + x (x fastest), N = nx*ny*nz.
 *   - Host arrays are caller-owned; the library copies what it needs and never
 *     keeps a host pointer after a call returns.
 *   - "Canonical populations" are FP64 host arrays f[(s*19 + i)*N + n] holding
 *     the pre-collision state f_i(x, t) of Eq. (LGS) at the current time t.
 *   - Every function returns LBM_OK (0) or a negative LBM_E* code; on error
 *     nothing is modified unless stated.
 *   - Calls on one context are not thread-safe; distinct contexts are
 *     independent.  Work is queued on the context's HIP stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_OK 0
#define LBM_EINVAL (-1)    /* invalid argument or parameter               */
#define LBM_ENOMEM (-2)    /* allocation failed / does not fit the budget */
#define LBM_EDEVICE (-3)   /* HIP runtime error or no usable device       */
#define LBM_EUNSTABLE (-4) /* non-finite state found by the health check  */
#define LBM_ENOTFOUND (-5) /* unknown ticket                              */
#define LBM_EAGAIN (-6)    /* result not ready yet                        */

#define LBM_MAX_RES 4

/* Storage format of the populations.  Arithmetic is FP64 for LBM_F64 and FP32
 * otherwise.  Stored value h = (f_i - w_i*rho_shift[s]) * 2^store_scale_log2,
 * rounded as lbm_params.rounding says for the 16-bit formats. */
typedef enum {
    LBM_F64 = 0,
    LBM_F32 = 1,
    LBM_F16S = 2,  /* IEEE binary16, shifted   */
    LBM_BF16S = 3  /* bfloat16, shifted        */
} lbm_storage;

/* Rounding of the 16-bit formats (FP32 and FP64 always round to nearest).
 * Stochastic rounding takes the upper neighbour with probability equal to the
 * dropped fraction, so it is unbiased: changes smaller than half a unit in the
 * last place survive on average instead of being rounded away every step (a
 * slowly developing flow otherwise stalls short of its steady state).  Its
 * random bits are a hash (MurmurHash3 32-bit finaliser) of the cell index,
 * component, direction and time step, so results are reproducible bit for bit
 * and do not depend on the launch decomposition. */
typedef enum {
    LBM_ROUND_NEAREST = 0,   /* round to nearest, ties to even */
    LBM_ROUND_STOCHASTIC = 1
} lbm_rounding;

/* Collision and forcing scheme.  LBM_FORCING_SHAN_CHEN is the HMCSC of
 * Eq. (HMCSC) / Eq. (LGS): the forces enter through the force-shifted
 * equilibrium velocity of Eq. (SC_u_eq).  LBM_FORCING_GUO is the grayscale
 * scheme the paper contrasts it with (appendix on Guo vs. Shan-Chen forcing,
 * Eq. GS-WBS): equilibrium at u_macro of Eq. (HMCSC_u_macro) plus (1 - n_s)
 * times the forcing term of Guo, Zheng and Shi (2002).  The GS-WBS runs with
 * the default tile shapes and is not accepted by the batched server. */
typedef enum {
    LBM_FORCING_SHAN_CHEN = 0,
    LBM_FORCING_GUO = 1
} lbm_forcing;

typedef struct {
    int32_t nx, ny, nz;
} lbm_domain;

/* Density reservoir (Sec. 4; Sec. 3.4 prescribes densities at the inlet and
 * outlet): cells with lo <= coordinate[axis] < hi have their pre-collision
 * state reset to the rest equilibrium w_i*rho[s] of Eq. (Maxwell) every step,
 * before the moments are taken. */
typedef struct {
    int32_t axis; /* 0: x, 1: y, 2: z */
    int32_t lo, hi;
    int32_t pad;
    double rho[2];
} lbm_reservoir;

typedef struct {
    int32_t ncomp;            /* 1 or 2 fluid components                               */
    int32_t c_ns;             /* 1: one n_s field for all components; 2: one per component */
    double tau[2];            /* relaxation times, > 0.5 (Eq. LGS; nu = (tau - 1/2)/3)  */
    double G_inter;           /* G_inter,12 = G_inter,21 of Eq. (SC_F_inter)            */
    double G_ads[2];          /* G_ads,sigma of Eq. (SC_F_ads)                          */
    double F_ext[3];          /* external force density, split by Eq. (SC_F_ext)        */
    double g_scale;           /* interaction stencils weight neighbours by g_scale*w_i;
                                 1 is the paper's Eqs. (SC_F_inter), (SC_F_ads)          */
    double rho_shift[2];      /* rho0_sigma of the shifted storage                      */
    int32_t storage;          /* lbm_storage                                            */
    int32_t store_scale_log2; /* power-of-two scale of stored values (16-bit formats)   */
    int32_t n_res;            /* number of reservoirs, 0..LBM_MAX_RES                   */
    int32_t check_every;      /* health check (finite mass) every k steps; 0 = never    */
    int32_t rounding;         /* lbm_rounding (16-bit formats)                          */
    int32_t forcing;          /* lbm_forcing                                            */
    lbm_reservoir res[LBM_MAX_RES];
} lbm_params;

/* Device memory a context needs, for callers that allocate it themselves. */
typedef struct {
    uint64_t pop_bytes;     /* each of the two population buffers            */
    uint64_t ns_bytes;      /* bounce-back fractions (float32, c_ns*N)        */
    uint64_t scratch_bytes; /* moments, checkpoint staging and reductions     */
} lbm_sizes;

/* Caller-provided device buffers (e.g. from PyTorch).  All four must be given,
 * 256-byte aligned, of at least the sizes of lbm_required_bytes, and must
 * outlive the context.  The library never frees them. */
typedef struct {
    void* f_a;
    void* f_b;
    void* n_s;
    void* scratch;
} lbm_device_buffers;

typedef struct {
    double mass[2];     /* sum over cells of rho_sigma (Eq. rho_BGK), FP64      */
    double momentum[3]; /* sum over cells of rho*u_macro (Eq. HMCSC_u_macro)    */
    int64_t time;       /* time step t of the state the totals describe         */
    int32_t finite;     /* 1 if every mass and momentum total is finite         */
    int32_t pad;
} lbm_totals;

typedef struct lbm_ctx lbm_ctx;

/* Size of each device buffer for the domain and parameters.  LBM_EINVAL when the
 * parameters are rejected (same rules as lbm_create). */
int lbm_required_bytes(const lbm_domain* dom, const lbm_params* prm, lbm_sizes* out);

/* Create a simulation and initialise it at t = 0 to the rest equilibrium
 * f_i = w_i*rho_init[s*N + n] (u = 0) of Eq. (Maxwell); reservoir cells start at
 * their prescribed densities.
 *   n_s      float32 host array [c_ns][N], every value in [0, 1] (Eq. LGS).
 *   rho_init FP64 host array [ncomp][N], finite.
 *   bufs     caller device buffers, or NULL: the library allocates and frees them.
 *   stream   hipStream_t to queue all work on, or NULL for the default stream.
 * Rejects ncomp/c_ns outside {1,2} (c_ns <= ncomp), tau <= 0.5, n_s outside
 * [0,1], empty or over-large domains, bad reservoirs or storage (LBM_EINVAL).
 * *out is NULL on failure.  Returns after the initial state is queued. */
int lbm_create(const lbm_domain* dom, const float* n_s, const double* rho_init,
               const lbm_params* prm, const lbm_device_buffers* bufs, void* stream,
               lbm_ctx** out);

/* Advance nsteps >= 0 time steps, asynchronously on the context stream.  When
 * check_every > 0 the FP64 totals are checked every check_every steps (this
 * synchronises) and LBM_EUNSTABLE is returned, with the time of the failing
 * check kept, if they are not finite. */
int lbm_step(lbm_ctx* ctx, int64_t nsteps);

/* Macroscopic fields at the current time t, from the pre-collision state,
 * computed on the device in FP64 and copied to caller-owned host arrays (any
 * pointer may be NULL):
 *   rho [ncomp][N]  rho_sigma, Eq. (rho_BGK)
 *   u   [3][N]      u_macro, Eq. (HMCSC_u_macro), with F_tot of Sec. 2
 *   p   [N]         p = (rho + g_scale*G_inter*rho_1*rho_2)/3, Eq. (SC_pressure)
 *   tot             FP64 totals (lbm_totals)
 * Synchronises the context stream. */
int lbm_moments(lbm_ctx* ctx, double* rho, double* u, double* p, lbm_totals* tot);

/* FP64 totals only (no per-cell copy-back).  Synchronises. */
int lbm_totals_get(lbm_ctx* ctx, lbm_totals* tot);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the FP64
 * totals of lbm_totals_get, computed in one pass that keeps no per-cell field
 * (each cell recomputes its neighbours' densities), with the per-block partial
 * sums in a fixed 82 KB device array of the library (2048 blocks x 5 doubles
 * plus the totals), one per device, held until the process ends.  It
 * allocates nothing and does not touch the context's scratch buffer; any
 * domain the context accepts fits (the grid strides over the cells with at
 * most 2048 blocks).  The totals equal lbm_totals_get's up to the order of the
 * FP64 sums.  Calls that overlap on one device share its array and race:
 * serialise them.  Synchronises the context stream; LBM_EINVAL for NULL
 * arguments, LBM_EDEVICE if the array cannot be located or a launch fails. */
int lbm_totals_get_static(lbm_ctx* ctx, lbm_totals* tot);

/* Electrolyte-filling diagnostics of Sec. 4, on slabs lo <= coordinate[axis]
 * < hi of the current (pre-collision) state at time t:
 *   capillary pressure, Eq. (CapPressure): dp = <p>_inlet - <p>_outlet, the
 *     means of the pressure of Eq. (SC_pressure) over the inlet and outlet
 *     slabs (typically the two reservoirs);
 *   saturation, Eq. (Saturation), of component comp over the pore slab (the
 *     cells between the membranes):
 *     S = sum (1 - n_s) [rho_comp >= threshold] / sum (1 - n_s),
 *     so resolved pore cells (n_s = 0) count once, homogenized cells with
 *     their fluid fraction 1 - n_s and solid cells (n_s = 1) not at all; n_s
 *     is component comp's own field when c_ns = 2.  The paper's threshold is
 *     0.5 mu/lu^3.
 * FP64, deterministic (fixed-order reduction).  Synchronises.  LBM_EINVAL for
 * an axis outside 0..2, comp >= ncomp, an empty or out-of-range inlet or
 * outlet slab, or a pore slab outside the domain.  S is 0 when the pore slab
 * holds no fluid volume. */
typedef struct {
    int32_t axis;                 /* 0: x, 1: y, 2: z                       */
    int32_t inlet_lo, inlet_hi;
    int32_t outlet_lo, outlet_hi;
    int32_t pore_lo, pore_hi;
    int32_t comp;                 /* component whose saturation is reported */
    double threshold;             /* density threshold of Eq. (Saturation)  */
} lbm_fill_query;

typedef struct {
    double dp;           /* <p>_inlet - <p>_outlet             */
    double p_inlet;
    double p_outlet;
    double saturation;   /* S of component comp                */
    double pore_volume;  /* sum of (1 - n_s) over the pore slab */
    int64_t time;
} lbm_fill_state;

int lbm_fill_state_get(lbm_ctx* ctx, const lbm_fill_query* q, lbm_fill_state* out);

/* Permeability of Eq. (Permeability) along axis (0: x, 1: y, 2: z) at the
 * current time t (Sec. 3.1): k = nu <rho u> / F, with <rho u> the mean over
 * all N cells of rho u_macro[axis] (Eq. HMCSC_u_macro, the momentum that
 * lbm_totals sums), F = F_ext[axis] of the context's parameters and
 * nu = (tau - 1/2)/3 the lattice viscosity.  k_comp[s] = nu <rho_s
 * u_macro[axis]> / F is component s's share (the mixture velocity weighted by
 * that component's density; k_comp[0] + k_comp[1] = k); its ratio to the
 * value of a run saturated with component s is the relative permeability of
 * Eq. (relativePermeability).  The run should be at steady state; k is
 * whatever the current state gives.  FP64, deterministic (fixed-order
 * reduction).  Synchronises.  LBM_EINVAL for NULL arguments, an axis outside
 * 0..2, F_ext[axis] = 0, or two components with different tau (no single
 * viscosity). */
typedef struct {
    double k;            /* nu <rho u> / F                              */
    double k_comp[2];    /* nu <rho_s u> / F (k_comp[1] = 0 if ncomp 1) */
    double momentum;     /* <rho u_macro[axis]>, mean over the cells    */
    double nu;           /* (tau - 1/2)/3                               */
    int64_t time;
} lbm_permeability;

int lbm_permeability_get(lbm_ctx* ctx, int32_t axis, lbm_permeability* out);

/* Static-droplet measurement of Sec. 3.3 (Laplace's law), FP64 on the device,
 * from the current pre-collision state.  For a droplet (or bubble) of
 * component comp centred at center (lattice coordinates; distances to the
 * nearest periodic image of the centre):
 *   rho_in  = mean rho_comp over |x - c| <= r_core (the bulk inside),
 *   rho_out = mean rho_comp over |x - c| >= r_far (the bulk outside),
 *   R       = radius of the volume V = (M_comp - rho_out N) / (rho_in -
 *             rho_out), M_comp the component's mass: a ball in 3-D,
 *             R = (3 V / (4 pi))^(1/3), a disc when nz = 1, R = (V / pi)^(1/2),
 *   p_in    = mean pressure of Eq. (SC_pressure) over |x - c| <= R / 2,
 *   p_out   = mean pressure over |x - c| >= R + margin,
 *   dp      = p_in - p_out, and gamma = dp R / 2 in 3-D, dp R in 2-D (the
 *             interfacial tension by Laplace's law).
 * Synchronises.  LBM_EINVAL for NULL arguments, comp >= ncomp, a non-finite
 * centre, r_core <= 0, r_far <= r_core, margin < 0, an empty averaging region,
 * or no droplet (rho_in = rho_out, or V <= 0). */
typedef struct {
    double center[3];
    double r_core, r_far;   /* radii of the inner and outer bulk samples */
    double margin;          /* p_out is taken beyond R + margin          */
    int32_t comp;
    int32_t pad;
} lbm_droplet_query;

typedef struct {
    double R, dp, gamma;
    double p_in, p_out;
    double rho_in, rho_out;
    int64_t time;
} lbm_droplet_state;

int lbm_droplet_get(lbm_ctx* ctx, const lbm_droplet_query* q, lbm_droplet_state* out);

/* Canonical populations (see above) of the current state into f [ncomp*19*N].
 * Reservoir cells hold their prescribed equilibrium.  Synchronises. */
int lbm_get_populations(lbm_ctx* ctx, double* f);

/* Replace the state by canonical populations f [ncomp*19*N] (rounded to
 * nearest in the storage format).  The time counter is kept.  Synchronises. */
int lbm_set_populations(lbm_ctx* ctx, const double* f);

/* Set the time counter (t >= 0), e.g. to resume a checkpoint taken at time t:
 * stochastic rounding draws on the time step, so a resumed run repeats the
 * original bit for bit only from the same t. */
int lbm_set_time(lbm_ctx* ctx, int64_t t);

/* Change the prescribed densities of reservoir r (e.g. a rising inlet density,
 * Sec. 4) from the next step on. */
int lbm_set_reservoir(lbm_ctx* ctx, int32_t r, const double rho[2]);

/* Current time step t (number of steps applied since creation). */
int64_t lbm_time(const lbm_ctx* ctx);

/* Block until all queued work of the context is done. */
int lbm_sync(lbm_ctx* ctx);

/* Average device time in milliseconds of the step kernel launches of the last
 * lbm_step call, measured with HIP events on the context stream (0 if none). */
double lbm_last_step_ms(const lbm_ctx* ctx);

/* Free library-owned memory (bound buffers are left alone).  Synchronises.
 * NULL is ignored. */
void lbm_destroy(lbm_ctx* ctx);

/* Static text for an LBM_E* code. */
const char* lbm_strerror(int code);

/* ---------------------------------------------------------------------------
 * Batched stepping: many domains, one kernel launch per step.
 *
 * A group steps a fixed set of contexts together; each launch runs the update
 * of every domain (same storage format, component count and n_s count) over a
 * device table of domains, so small domains share the GPU instead of each
 * paying a launch.  Results are bitwise those of lbm_step on each context.
 */
typedef struct lbm_group lbm_group;

/* Group the n contexts ctxs[0..n-1] (caller keeps ownership; they must
 * outlive the group and not be stepped on their own meanwhile).  Work is
 * queued on the stream of ctxs[0].  LBM_EINVAL if they differ in storage,
 * ncomp or c_ns, if any uses LBM_FORCING_GUO, or n < 1. */
int lbm_group_create(lbm_ctx* const* ctxs, int32_t n, lbm_group** out);

/* Advance every context of the group by nsteps (asynchronous; launches are
 * replayed from a captured HIP graph).  Each context's time advances. */
int lbm_group_step(lbm_group* g, int64_t nsteps);

/* Average device time in ms of one batched launch of the last lbm_group_step. */
double lbm_group_last_step_ms(const lbm_group* g);

void lbm_group_destroy(lbm_group* g);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of simulation requests.
 *
 * A server owns a worker thread and three streams (ticks, admissions,
 * retirements; default priority).  Requests (domain, n_s, initial densities,
 * parameters, step budget, convergence test) are queued by lbm_batch_submit
 * from any thread.  The worker admits queued requests in arrival order while
 * a slot is free and the resident state fits the HBM budget: their state gets
 * a block of a device memory pool (grown in chunks up to the budget and kept),
 * their arrays are uploaded and the state initialised on the admission
 * stream while ticks run.  A tick replays a captured graph of steps_per_tick
 * batched launches over the resident domains its policy steps (a domain that
 * needs fewer steps stops early) and, for the domains with a convergence
 * test, one batched FP64 reduction of their momentum.  Ticks are not waited
 * for: the worker launches tick k, then reads tick k-1's reductions and
 * retires what tick k-1 finished, while tick k runs.  A request whose test
 * fires on tick k's state is therefore stepped by tick k+1 too (always
 * exactly one tick more, alone or in a mix), and stops after it.  Each result
 * is the same as running the request alone for the same number of steps.
 */
typedef struct lbm_server lbm_server;

/* How a tick's launches are shared among the resident domains.  FAIR steps
 * every resident domain each tick (processor sharing).  SHORTEST_FIRST steps
 * only the domains with the least remaining work, cells x (max_steps -
 * steps_done), smallest first, until the stepped set holds run_cells cells;
 * the others wait with their state untouched.  It lowers mean completion time
 * when short and long requests mix; a long request waits while shorter ones
 * keep arriving and fill run_cells, and the convergence test of a request
 * runs only on the ticks that step it. */
typedef enum {
    LBM_SERVE_FAIR = 0,
    LBM_SERVE_SHORTEST_FIRST = 1
} lbm_serve_policy;

typedef struct {
    uint64_t hbm_budget_bytes; /* resident population + n_s bytes; 0: 90 % of free device memory */
    int32_t max_slots;         /* domains resident at once (>= 1)                            */
    int32_t steps_per_tick;    /* launches per graph replay and between checks (>= 1)         */
    int32_t storage;           /* lbm_storage of every request                               */
    int32_t ncomp, c_ns;       /* component and n_s-field counts of every request            */
    int64_t max_cells;         /* largest accepted domain (sizes the shared scratch)         */
    int32_t tile_x, tile_y;    /* tile of the batched kernel; 0: 64 x 8                      */
    int32_t policy;            /* lbm_serve_policy                                           */
    int32_t pad;               /* must be 0                                                  */
    int64_t run_cells;         /* SHORTEST_FIRST: cells stepped per tick at least; 0: 2^24   */
} lbm_server_cfg;

typedef struct {
    lbm_domain dom;
    const float* n_s;         /* [c_ns][N], copied at submit                                 */
    const double* rho_init;   /* [ncomp][N], copied at submit                                */
    lbm_params params;        /* storage, ncomp and c_ns must match the server               */
    int64_t max_steps;        /* run at most this many steps (>= 1)                          */
    double conv_tol;          /* convergence test on the state after each tick, 0 disables.
                                 Sample: J = sum over cells of sum_s (1 - n_s)(j_s + F_ext,s/2),
                                 the mixture momentum of Eq. (HMCSC_u_macro) without the
                                 neighbour forces, FP64 on the device.  conv_window <= 1:
                                 stop when |J(t) - J(t-K)| <= conv_tol |J(t)| (K =
                                 steps_per_tick).  conv_window = W > 1: stop when the means of
                                 the last two windows of W samples differ by at most conv_tol
                                 times the newer one                                          */
    int32_t conv_window;      /* samples per window, 0..1024 (0 and 1: consecutive samples)  */
    int32_t conv_noise;       /* 1: with W > 1, also stop when the two window means differ by
                                 at most twice the standard error of their difference (from
                                 the spread within the windows): the state no longer drifts
                                 beyond its own rounding noise.  A stochastically rounded
                                 16-bit state carries noise of order 1e-4..1e-2 in J, far above
                                 a tolerance of 1e-6, which alone would then never be met    */
    double* rho_out;          /* optional caller buffer [ncomp][N] for the final densities;
                                 must stay valid until the result is final                   */
} lbm_request;

typedef struct {
    int32_t status;       /* LBM_OK or the error that ended the request   */
    int32_t converged;    /* 1 if stopped by the convergence test          */
    int64_t steps_done;
    double t_submit;      /* seconds on the server clock                    */
    double t_admit;
    double t_done;
    lbm_totals totals;    /* FP64 totals of the final state                 */
} lbm_result;

typedef struct {
    int64_t submitted, completed, queued, active;
    double cell_updates;   /* cell updates executed (all domains)        */
    double busy_seconds;   /* time with at least one resident domain      */
    double uptime_seconds;
    uint64_t bytes_resident;
    int64_t ticks;
} lbm_server_stats;

/* Create a server on the current device.  reserved must be NULL. */
int lbm_server_create(const lbm_server_cfg* cfg, void* reserved, lbm_server** out);

/* Queue a request; *ticket identifies it.  LBM_EINVAL for invalid input
 * (including conv_window outside 0..1024, conv_noise not 0 or 1, non-finite
 * densities), a format mismatch or LBM_FORCING_GUO, LBM_ENOMEM if its state can
 * never fit the budget or it exceeds max_cells.  Thread-safe. */
int lbm_batch_submit(lbm_server* s, const lbm_request* req, uint64_t* ticket);

/* Result of a ticket: LBM_OK and *out filled when final, LBM_EAGAIN while
 * queued or running, LBM_ENOTFOUND for an unknown ticket.  Thread-safe. */
int lbm_batch_poll(lbm_server* s, uint64_t ticket, lbm_result* out);

/* Like lbm_batch_poll but blocks up to timeout_s seconds (< 0: forever). */
int lbm_batch_wait(lbm_server* s, uint64_t ticket, double timeout_s, lbm_result* out);

int lbm_server_stats_get(lbm_server* s, lbm_server_stats* out);

/* Stop the worker (queued and running requests end with LBM_EAGAIN status),
 * free all device memory.  NULL is ignored. */
void lbm_server_destroy(lbm_server* s);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
