// Internal interface between the host runtime and the HIP kernels of the HMCSC
// library.  Not part of the public ABI (that is include/lbm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hm {

constexpr int kQ = 19;
constexpr int kMaxRes = 4;
constexpr int kForcingShanChen = 0;  // Eq. (HMCSC)
constexpr int kForcingGuo = 1;       // Eq. (GS-WBS)

enum Storage { kF64 = 0, kF32 = 1, kF16 = 2, kBF16 = 3 };

// Everything a launch needs besides the buffers, in double precision; the
// launchers convert to the arithmetic type of the storage format.
struct Problem {
    int nx, ny, nz;
    int64_t N;
    int ncomp, c_ns;
    int storage;
    double tau[2];
    double G_s;        // G_inter * g_scale
    double Gads_s[2];  // G_ads * g_scale
    double F[3];
    double rho0[2];
    double scale;      // 2^store_scale_log2
    int stochastic;    // 16-bit formats: stochastic rounding of stored values
    int forcing;       // kForcingShanChen (the HMCSC) or kForcingGuo (the GS-WBS)
    double g_scale, G_inter;
    int n_res;
    int res_axis[kMaxRes], res_lo[kMaxRes], res_hi[kMaxRes];
    double res_rho[kMaxRes][2];
};

struct Launch {
    int tile_x;   // cells per tile row (32, 64 or 128)
    int tile_y;   // rows per tile (split layout: 4 with 128-wide rows, 4 or 8 with 64, 4, 8
                  // or 16 with 32; pair layout: 4 or pair_tile_y() with 64)
    int zchunk;   // planes per block
};

// True if two components in this format use the pair layout: both values of
// one (cell, direction) in one word (FP32 and the 16-bit formats; FP32 with
// the GS-WBS keeps the split layout), plane blocks [z][i][y][x][s]; all other
// runs use the split layout [s][z][i][y][x].
bool pair_layout(int storage, int ncomp, int forcing = kForcingShanChen);

// Rows of the default tile of the pair kernel (64 cells wide).
int pair_tile_y();

// True if the tile shape is compiled in for this format, component count and
// forcing scheme.
bool tile_supported(int storage, int ncomp, int tile_x, int tile_y, int forcing = kForcingShanChen);

// Bytes per stored population.
int storage_bytes(int storage);

// One time step A -> B (pull streaming, fused forces/collision/bounce-back);
// t is the time step of the state in A (keys the stochastic rounding).
hipError_t launch_step(const Problem& p, const Launch& l, int64_t t, const void* A, void* B,
                       const float* ns, hipStream_t s);

// t = 0 state: rest equilibrium of rho_init (device FP64 [ncomp][N]).
hipError_t launch_init(const Problem& p, const double* rho_init, void* A, hipStream_t s);

// Canonical FP64 pre-collision populations of component/direction (s, i)
// into out[N] (pull + decode + reservoir reset).
hipError_t launch_canonical(const Problem& p, const void* A, int s, int i, double* out,
                            hipStream_t st);

// Store canonical FP64 populations of (s, i) from in[N] into A.
hipError_t launch_set_canonical(const Problem& p, const double* in, int s, int i, void* A,
                                hipStream_t st);

// FP64 diagnostics of the state in A: densities rho [ncomp][N] (always),
// u_macro [3][N] and p [N] when not NULL, and the totals out[5] = {M_0, M_1,
// J_x, J_y, J_z} with J = sum rho u_macro, deterministic (fixed-order
// reductions).  With forces false only the first pass runs: rho and the
// local part of J, sum (1 - n_s)(j + F_ext/2), enough for a health check;
// u and p need forces.  partials holds 10 * moments_max_blocks() doubles.
hipError_t launch_diagnostics(const Problem& p, const void* A, const float* ns, bool forces, double* rho,
                              double* u, double* pr, double* partials, double* out, hipStream_t st);

int moments_max_blocks();

// The totals of launch_diagnostics (forces included) in one pass that keeps
// no per-cell field: partial sums of at most max_blocks blocks (5 doubles
// each) in partials, the totals in out[5].
hipError_t launch_totals_one_pass(const Problem& p, const void* A, const float* ns, double* partials, int max_blocks,
                                  double* out, hipStream_t st);

// Slabs of the filling diagnostics (Sec. 4), coordinates along axis.
struct FillQuery {
    int axis;
    int inlet_lo, inlet_hi, outlet_lo, outlet_hi, pore_lo, pore_hi;
    int comp;
    double threshold;
};

// Eq. (CapPressure) and Eq. (Saturation) sums from the FP64 densities rho and
// pressure pr: out[6] = {sum p inlet, cells inlet, sum p outlet, cells outlet,
// sum (1-n_s)[rho_comp >= threshold] pore, sum (1-n_s) pore}.  partials needs
// 6 * moments_max_blocks() doubles.
hipError_t launch_fill(const Problem& p, const FillQuery& q, const double* rho, const double* pr, const float* ns,
                       double* partials, double* out, hipStream_t st);

// Static-droplet sums (Sec. 3.3) of the FP64 field f [N]: out[4] = {sum f
// over |x - c| <= r_in, cells there, sum f over |x - c| >= r_out, cells
// there}, distances to the nearest periodic image of c.  partials needs
// 4 * moments_max_blocks() doubles.
hipError_t launch_ball(const Problem& p, const double c[3], double r_in, double r_out, const double* f,
                       double* partials, double* out, hipStream_t st);

// Eq. (Permeability) sums from the FP64 densities rho and velocity u (after
// the force pass): out[3] = {sum rho_0 u[axis], sum rho_1 u[axis], sum rho
// u[axis]}.  partials needs 3 * moments_max_blocks() doubles.
hipError_t launch_flux(const Problem& p, int axis, const double* rho, const double* u, double* partials, double* out,
                       hipStream_t st);

// One domain of a batched launch (host description).
struct BatchDomain {
    Problem prob;
    int zchunk;
    const void* buf[2];  // population buffers (ping-pong)
    const float* ns;
    int parity;          // buffer holding the state before the first launch of the tick
    int64_t t;           // time step of that state
    int steps;           // launches k = 0 .. steps-1 of the tick advance this domain
};

// Size of a device table for up to max_domains domains.
size_t batch_table_bytes(int storage, int max_domains);

// Encode the table for n domains into host memory (batch_table_bytes bytes);
// returns the total number of tiles.  Upload it to the device before launching.
int batch_encode(int storage, const BatchDomain* d, int n, int tile_x, int tile_y, void* host);

// Tile shapes compiled for the batched kernel, and the default one.
bool batch_tile_supported(int storage, int ncomp, int tile_x, int tile_y);
void batch_default_tile(int storage, int ncomp, int* tile_x, int* tile_y);

// Blocks of the batched kernel that fit one CU at once (registers, LDS); at
// least 1.
int batch_blocks_per_cu(int storage, int ncomp, int c_ns, int tile_x, int tile_y);

// Launch k of a tick: every domain with k < steps takes one step.  The grid
// strides over all tiles of the table, so any fixed grid size works.
hipError_t launch_step_batch(int storage, int ncomp, int c_ns, int tile_x, int tile_y, const void* table, int k,
                             int grid, hipStream_t st);

// Convergence monitor (server): one domain of a monitor table.
struct MonitorDomain {
    Problem prob;
    const void* state;  // buffer holding the state to monitor
    const float* ns;
};

constexpr int kMonitorBlocksPerDomain = 256;

// Size of a device monitor table for up to max_domains domains, and the
// most blocks (partials of 4 doubles each) its launch uses.
size_t monitor_table_bytes(int storage, int max_domains);
int monitor_max_blocks(int max_domains);

// Encode the table for n domains into host memory; returns the total number
// of blocks of the launch.
int monitor_encode(int storage, const MonitorDomain* d, int n, void* host);

// For each domain d of the (device) table: out[4 d .. 4 d + 3] = {sum over
// cells of sum_s (1 - n_s)(j_s + F_ext,s / 2) (x, y, z), sum of rho}, FP64,
// deterministic.  partials holds 4 * total_blocks doubles.
hipError_t launch_monitor(int storage, const void* table, int ndom, int total_blocks, double* partials, double* out,
                          hipStream_t st);

}  // namespace hm
