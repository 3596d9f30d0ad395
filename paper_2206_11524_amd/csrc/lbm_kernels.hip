// HIP kernels (gfx950) of the HMCSC lattice Boltzmann update.
//
// Layout in HBM: populations are structure-of-arrays, P[(s*19 + i)*N + n] with
// n = (z*ny + y)*nx + x.  Streaming is "pull": a buffer holds the populations
// that left each cell at the previous step, so the pre-collision state of
// Eq. (LGS) at cell x is f_i(x) = P_i(x - c_i) (periodic).  Every stored value is
// shifted, h = f - w_i*rho0_s (scaled by 2^k for the 16-bit formats); the whole
// collision is written in the shifted variables (the shift cancels in the
// partial bounce-back blend because w_ibar = w_i), which keeps small deviations
// representable in reduced precision.
//
// The step kernel is a fused 2.5-D sweep: a block owns a 64 x TY column of
// cells and marches along z.  For every plane it pulls the populations of its
// cells once (kept in registers for the collision of the next iteration),
// forms the densities, and stages them in LDS together with a one-cell ring of
// densities recomputed from the ring cells' populations, plus the n_s field.
// The cohesion force (Eq. SC_F_inter) and adhesion force (Eq. SC_F_ads) then
// read their 18 neighbours from LDS, so HBM sees each population read once
// and written once per step (ring and z-halo re-reads hit L2/MALL).
#include "lbm_kernels.h"

#include <stdint.h>

namespace hm {

// ---------------------------------------------------------------------------
// D3Q19 velocity set, ordered as printed in Appendix A: directions i and i+9
// (i = 1..9) are opposite.  Weights 1/3, 1/18 (|c| = 1), 1/36 (|c| = sqrt 2).
__device__ constexpr int CX[kQ] = {0, -1, 0, 0, -1, -1, -1, -1, 0, 0, 1, 0, 0, 1, 1, 1, 1, 0, 0};
__device__ constexpr int CY[kQ] = {0, 0, -1, 0, -1, 1, 0, 0, -1, -1, 0, 1, 0, 1, -1, 0, 0, 1, 1};
__device__ constexpr int CZ[kQ] = {0, 0, 0, -1, 0, 0, -1, 1, -1, 1, 0, 0, 1, 0, 0, 1, -1, 1, -1};

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : (i <= 9 ? i + 9 : i - 9); }

template <typename T>
__host__ __device__ constexpr T wgt(int i)
{
    return i == 0 ? T(1) / T(3)
                  : ((CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i]) == 1 ? T(1) / T(18) : T(1) / T(36));
}

// ---------------------------------------------------------------------------
// Storage formats.  decode() returns the shifted value h in the arithmetic
// type T, encode() rounds h back (round to nearest even for 16-bit).
struct F64 {
    using E = double;
    using T = double;
    static __device__ __forceinline__ T dec(E v, T) { return v; }
    static __device__ __forceinline__ E enc(T v, T) { return v; }
};
struct F32 {
    using E = float;
    using T = float;
    static __device__ __forceinline__ T dec(E v, T) { return v; }
    static __device__ __forceinline__ E enc(T v, T) { return v; }
};
struct F16 {
    using E = uint16_t;
    using T = float;
    static __device__ __forceinline__ T dec(E v, T inv_scale)
    {
        return static_cast<float>(__builtin_bit_cast(_Float16, v)) * inv_scale;
    }
    static __device__ __forceinline__ E enc(T v, T scale)
    {
        return __builtin_bit_cast(uint16_t, static_cast<_Float16>(v * scale));
    }
};
struct BF16 {
    using E = uint16_t;
    using T = float;
    static __device__ __forceinline__ T dec(E v, T inv_scale)
    {
        return __uint_as_float(static_cast<uint32_t>(v) << 16) * inv_scale;
    }
    static __device__ __forceinline__ E enc(T v, T scale)
    {
        uint32_t u = __float_as_uint(v * scale);
        if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return static_cast<E>((u >> 16) | 0x40u);
        u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest, ties to even
        return static_cast<E>(u >> 16);
    }
};

// Kernel parameters in the arithmetic type.
template <typename T>
struct Args {
    int nx, ny, nz;
    int N;
    int zchunk, ntx, nty, nzc;
    T inv_tau[2], tau[2];
    T G_s, Gads_s[2];
    T F[3];
    T rho0[2];
    T scale, inv_scale;
    int n_res;
    int res_axis[kMaxRes], res_lo[kMaxRes], res_hi[kMaxRes];
    T res_dr[kMaxRes][2];  // rho_res - rho0, shifted density of the reservoir
};

template <typename T>
static Args<T> make_args(const Problem& p)
{
    Args<T> a{};
    a.nx = p.nx; a.ny = p.ny; a.nz = p.nz;
    a.N = static_cast<int>(p.N);
    for (int s = 0; s < 2; ++s) {
        a.tau[s] = static_cast<T>(p.tau[s]);
        a.inv_tau[s] = static_cast<T>(1.0 / p.tau[s]);
        a.Gads_s[s] = static_cast<T>(p.Gads_s[s]);
        a.rho0[s] = static_cast<T>(p.rho0[s]);
    }
    a.G_s = static_cast<T>(p.G_s);
    for (int d = 0; d < 3; ++d) a.F[d] = static_cast<T>(p.F[d]);
    a.scale = static_cast<T>(p.scale);
    a.inv_scale = static_cast<T>(1.0 / p.scale);
    a.n_res = p.n_res;
    for (int r = 0; r < kMaxRes; ++r) {
        a.res_axis[r] = p.res_axis[r];
        a.res_lo[r] = p.res_lo[r];
        a.res_hi[r] = p.res_hi[r];
        for (int s = 0; s < 2; ++s) a.res_dr[r][s] = static_cast<T>(p.res_rho[r][s] - p.rho0[s]);
    }
    return a;
}

template <typename T>
__device__ __forceinline__ int reservoir_of(const Args<T>& a, int x, int y, int z)
{
    int r_found = -1;
    for (int r = 0; r < kMaxRes; ++r) {
        if (r >= a.n_res) break;
        const int c = a.res_axis[r] == 0 ? x : (a.res_axis[r] == 1 ? y : z);
        if (r_found < 0 && c >= a.res_lo[r] && c < a.res_hi[r]) r_found = r;
    }
    return r_found;
}

__device__ __forceinline__ int wrap_dec(int v, int n) { return v == 0 ? n - 1 : v - 1; }
__device__ __forceinline__ int wrap_inc(int v, int n) { return v == n - 1 ? 0 : v + 1; }

// Source index of the pull for direction i at cell (x,y,z): the cell x - c_i.
// xs[0..2] = x+1, x, x-1 (index by 1 + c), same for rows and planes.
struct PullIdx {
    int col[3];   // x - c for c = -1, 0, +1  -> index c+1
    int row[3];   // (y - c) * nx
    int pln[3];   // (z - c) * nx * ny
};

__device__ __forceinline__ PullIdx pull_idx(int x, int y, int z, int nx, int ny, int nz)
{
    PullIdx q;
    q.col[0] = wrap_inc(x, nx); q.col[1] = x; q.col[2] = wrap_dec(x, nx);
    q.row[0] = wrap_inc(y, ny) * nx; q.row[1] = y * nx; q.row[2] = wrap_dec(y, ny) * nx;
    const int plane = nx * ny;
    q.pln[0] = wrap_inc(z, nz) * plane; q.pln[1] = z * plane; q.pln[2] = wrap_dec(z, nz) * plane;
    return q;
}

// Pull the shifted pre-collision populations of one cell and component.
template <typename ST, typename T>
__device__ __forceinline__ void pull_cell(const typename ST::E* __restrict__ A, const Args<T>& a,
                                          const PullIdx& q, int s, int res, T h[kQ])
{
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int src = q.pln[CZ[i] + 1] + q.row[CY[i] + 1] + q.col[CX[i] + 1];
        const typename ST::E* Ai = A + static_cast<size_t>(s * kQ + i) * static_cast<size_t>(a.N);
        h[i] = ST::dec(Ai[src], a.inv_scale);
    }
    if (res >= 0) {
        const T dr = a.res_dr[res][s];
#pragma unroll
        for (int i = 0; i < kQ; ++i) h[i] = wgt<T>(i) * dr;
    }
}

template <typename T>
__device__ __forceinline__ T sum19(const T h[kQ])
{
    // pairwise order, fixed
    T acc = h[0];
#pragma unroll
    for (int i = 1; i <= 9; ++i) acc += h[i] + h[i + 9];
    return acc;
}

// ---------------------------------------------------------------------------
// Fused step kernel.
template <typename ST, int NC, int CNS, int TY>
struct StepKernel {
    using T = typename ST::T;
    using E = typename ST::E;
    static constexpr int LW = kTileX + 2;       // LDS row width
    static constexpr int LP = LW * (TY + 2);    // LDS plane size
    static constexpr int NT = kTileX * TY;      // threads per block
};

template <typename ST, int NC, int CNS, int TY>
__global__ __launch_bounds__(kTileX* TY) void k_step(Args<typename ST::T> a,
                                                      const typename ST::E* __restrict__ A,
                                                      typename ST::E* __restrict__ B,
                                                      const float* __restrict__ ns)
{
    using K = StepKernel<ST, NC, CNS, TY>;
    using T = typename ST::T;
    using E = typename ST::E;
    constexpr int LW = K::LW, LP = K::LP, NT = K::NT;

    __shared__ T s_rho[3][NC][LP];
    __shared__ float s_ns[3][CNS][LP];

    // XCD-aware tile order: blocks are dispatched round-robin over 8 XCDs, so
    // give each XCD a contiguous run of tiles (neighbours share its L2).
    const int nb = gridDim.x;
    int L = blockIdx.x;
    if ((nb & 7) == 0) L = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
    const int tx = L % a.ntx;
    const int ty = (L / a.ntx) % a.nty;
    const int tz = L / (a.ntx * a.nty);
    const int x0 = tx * kTileX, y0 = ty * TY;
    const int zs = tz * a.zchunk;
    const int ze = min(zs + a.zchunk, a.nz);
    const int TXe = min(kTileX, a.nx - x0);
    const int TYe = min(TY, a.ny - y0);

    const int lx = threadIdx.x % kTileX;
    const int ly = threadIdx.x / kTileX;
    const bool act = lx < TXe && ly < TYe;
    const int x = x0 + min(lx, TXe - 1);
    const int y = y0 + min(ly, TYe - 1);
    const int me = (ly + 1) * LW + (lx + 1);

    // ring cell of this thread (if any): top row, bottom row, left, right column
    const int ring_n = 2 * (TXe + 2) + 2 * TYe;
    int rlx = 0, rly = 0;
    const bool ring = threadIdx.x < ring_n;
    {
        const int r = threadIdx.x;
        if (r < TXe + 2) { rlx = r - 1; rly = -1; }
        else if (r < 2 * (TXe + 2)) { rlx = r - (TXe + 2) - 1; rly = TYe; }
        else if (r < 2 * (TXe + 2) + TYe) { rlx = -1; rly = r - 2 * (TXe + 2); }
        else { rlx = TXe; rly = r - 2 * (TXe + 2) - TYe; }
    }
    const int rx = ((x0 + rlx) % a.nx + a.nx) % a.nx;
    const int ry = ((y0 + rly) % a.ny + a.ny) % a.ny;
    const int rme = (rly + 1) * LW + (rlx + 1);

    const int nsw = TXe + 2, nsh = TYe + 2;

    // Densities of plane p into LDS slot: own cell from registers (h), ring cells pulled.
    auto ring_density = [&](int p, int slot) {
        if (ring) {
            const PullIdx q = pull_idx(rx, ry, p, a.nx, a.ny, a.nz);
            const int res = reservoir_of(a, rx, ry, p);
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                T hh[kQ];
                pull_cell<ST, T>(A, a, q, s, res, hh);
                s_rho[slot][s][rme] = a.rho0[s] + sum19(hh);
            }
        }
    };
    auto load_ns = [&](int p, int slot) {
        const int plane = p * a.nx * a.ny;
        for (int k = threadIdx.x; k < nsw * nsh; k += NT) {
            const int llx = k % nsw - 1, lly = k / nsw - 1;
            const int gx = ((x0 + llx) % a.nx + a.nx) % a.nx;
            const int gy = ((y0 + lly) % a.ny + a.ny) % a.ny;
#pragma unroll
            for (int c = 0; c < CNS; ++c)
                s_ns[slot][c][(lly + 1) * LW + llx + 1] = ns[static_cast<size_t>(c) * a.N + plane + gy * a.nx + gx];
        }
    };
    auto wrapz = [&](int p) { return p < 0 ? p + a.nz : (p >= a.nz ? p - a.nz : p); };

    T cur[NC][kQ];
    T nxt[NC][kQ];

    // prologue: plane zs-1 (densities only) and plane zs (kept in cur)
    {
        const int pm = wrapz(zs - 1);
        if (act) {
            const PullIdx q = pull_idx(x, y, pm, a.nx, a.ny, a.nz);
            const int res = reservoir_of(a, x, y, pm);
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                pull_cell<ST, T>(A, a, q, s, res, nxt[s]);
                s_rho[0][s][me] = a.rho0[s] + sum19(nxt[s]);
            }
        }
        ring_density(pm, 0);
        load_ns(pm, 0);
        if (act) {
            const PullIdx q = pull_idx(x, y, zs, a.nx, a.ny, a.nz);
            const int res = reservoir_of(a, x, y, zs);
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                pull_cell<ST, T>(A, a, q, s, res, cur[s]);
                s_rho[1][s][me] = a.rho0[s] + sum19(cur[s]);
            }
        }
        ring_density(zs, 1);
        load_ns(zs, 1);
    }

    int sm = 0, s0 = 1, sp = 2;  // LDS slots of planes z-1, z, z+1
    for (int z = zs; z < ze; ++z) {
        const int pn = wrapz(z + 1);
        if (act) {
            const PullIdx q = pull_idx(x, y, pn, a.nx, a.ny, a.nz);
            const int res = reservoir_of(a, x, y, pn);
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                pull_cell<ST, T>(A, a, q, s, res, nxt[s]);
                s_rho[sp][s][me] = a.rho0[s] + sum19(nxt[s]);
            }
        }
        ring_density(pn, sp);
        load_ns(pn, sp);
        __syncthreads();

        if (act) {
            const int slot_of[3] = {sp, s0, sm};  // by 1 - c_z ... index with dz+1 below
            (void)slot_of;
            // moments
            T rho_s[NC], j[NC][3];
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                rho_s[s] = a.rho0[s] + sum19(cur[s]);
                T jx = 0, jy = 0, jz = 0;
#pragma unroll
                for (int i = 1; i < kQ; ++i) {
                    if (CX[i]) jx += CX[i] > 0 ? cur[s][i] : -cur[s][i];
                    if (CY[i]) jy += CY[i] > 0 ? cur[s][i] : -cur[s][i];
                    if (CZ[i]) jz += CZ[i] > 0 ? cur[s][i] : -cur[s][i];
                }
                j[s][0] = jx; j[s][1] = jy; j[s][2] = jz;
            }
            T rho = 0, den = 0, num[3] = {0, 0, 0};
#pragma unroll
            for (int s = 0; s < NC; ++s) {
                rho += rho_s[s];
                den += rho_s[s] * a.inv_tau[s];
#pragma unroll
                for (int d = 0; d < 3; ++d) num[d] += j[s][d] * a.inv_tau[s];
            }
            T up[3];
            const T inv_den = den > T(0) ? T(1) / den : T(0);
#pragma unroll
            for (int d = 0; d < 3; ++d) up[d] = num[d] * inv_den;
            const T inv_rho = rho > T(0) ? T(1) / rho : T(0);

#pragma unroll
            for (int s = 0; s < NC; ++s) {
                // neighbour stencils sum_i w_i phi(x + c_i) c_i from LDS
                T gi[3] = {0, 0, 0}, ga[3] = {0, 0, 0};
                const int cn = CNS == 2 ? s : 0;
#pragma unroll
                for (int i = 1; i < kQ; ++i) {
                    const int slot = CZ[i] == 0 ? s0 : (CZ[i] > 0 ? sp : sm);
                    const int k = me + CY[i] * LW + CX[i];
                    const T wi = wgt<T>(i);
                    if (NC == 2) {
                        const T r = s_rho[slot][1 - s][k] * wi;
                        if (CX[i]) gi[0] += CX[i] > 0 ? r : -r;
                        if (CY[i]) gi[1] += CY[i] > 0 ? r : -r;
                        if (CZ[i]) gi[2] += CZ[i] > 0 ? r : -r;
                    }
                    const T v = static_cast<T>(s_ns[slot][cn][k]) * wi;
                    if (CX[i]) ga[0] += CX[i] > 0 ? v : -v;
                    if (CY[i]) ga[1] += CY[i] > 0 ? v : -v;
                    if (CZ[i]) ga[2] += CZ[i] > 0 ? v : -v;
                }
                // force per unit density: F_tot,s / rho_s of Eqs. (SC_F_inter),
                // (SC_F_ads), (SC_F_ext); no shift for an absent component
                T ueq[3];
                const bool present = rho_s[s] > T(0);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const T acc = -a.G_s * gi[d] - a.Gads_s[s] * ga[d] + a.F[d] * inv_rho;
                    ueq[d] = up[d] + (present ? a.tau[s] * acc : T(0));
                }
                const T uu = ueq[0] * ueq[0] + ueq[1] * ueq[1] + ueq[2] * ueq[2];
                const T n = static_cast<T>(s_ns[s0][cn][me]);
                const T omn = T(1) - n;
                const T drho = rho_s[s] - a.rho0[s];
                E* Bs = B + static_cast<size_t>(s * kQ) * static_cast<size_t>(a.N);
                const int dst = (z * a.ny + y) * a.nx + x;
#pragma unroll
                for (int i = 0; i < kQ; ++i) {
                    const T cu = T(CX[i]) * ueq[0] + T(CY[i]) * ueq[1] + T(CZ[i]) * ueq[2];
                    const T heq = wgt<T>(i) * (drho + rho_s[s] * (cu * (T(3) + T(4.5) * cu) - T(1.5) * uu));
                    const T h = cur[s][i];
                    const T post = omn * (h - (h - heq) * a.inv_tau[s]) + n * cur[s][opp(i)];
                    Bs[static_cast<size_t>(i) * static_cast<size_t>(a.N) + dst] = ST::enc(post, a.scale);
                }
            }
        }
#pragma unroll
        for (int s = 0; s < NC; ++s)
#pragma unroll
            for (int i = 0; i < kQ; ++i) cur[s][i] = nxt[s][i];
        const int t = sm;
        sm = s0; s0 = sp; sp = t;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Auxiliary kernels (initialisation, checkpoints, FP64 diagnostics).  They run
// once per call, not per step, so they use a plain one-thread-per-cell grid.

template <typename ST>
__global__ void k_init(Args<typename ST::T> a, int ncomp, const double* __restrict__ rho_init,
                       typename ST::E* __restrict__ A)
{
    using T = typename ST::T;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
    const int x = n % a.nx, y = (n / a.nx) % a.ny, z = n / (a.nx * a.ny);
    // A_i(y) must hold f_i(y + c_i, 0) (pull storage)
    for (int s = 0; s < ncomp; ++s) {
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int xd = (x + CX[i] + a.nx) % a.nx, yd = (y + CY[i] + a.ny) % a.ny, zd = (z + CZ[i] + a.nz) % a.nz;
            const int d = (zd * a.ny + yd) * a.nx + xd;
            const int res = reservoir_of(a, xd, yd, zd);
            const double rho = res >= 0 ? static_cast<double>(a.res_dr[res][s]) + static_cast<double>(a.rho0[s])
                                        : rho_init[static_cast<size_t>(s) * a.N + d];
            const double h = wgt<double>(i) * (rho - static_cast<double>(a.rho0[s]));
            A[static_cast<size_t>(s * kQ + i) * a.N + n] = ST::enc(static_cast<T>(h), a.scale);
        }
    }
}

template <typename ST>
__global__ void k_canonical(Args<typename ST::T> a, const typename ST::E* __restrict__ A, int s, int i,
                            double* __restrict__ out)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
    const int x = n % a.nx, y = (n / a.nx) % a.ny, z = n / (a.nx * a.ny);
    const int res = reservoir_of(a, x, y, z);
    const int cxi = CX[0] * 0;  // silence unused warning patterns
    (void)cxi;
    int dx = 0, dy = 0, dz = 0;
    // runtime direction: small table walk
    for (int k = 0; k < kQ; ++k)
        if (k == i) { dx = CX[k]; dy = CY[k]; dz = CZ[k]; }
    double w = 0;
    for (int k = 0; k < kQ; ++k)
        if (k == i) w = wgt<double>(k);
    double v;
    if (res >= 0) {
        v = w * (static_cast<double>(a.res_dr[res][s]) + static_cast<double>(a.rho0[s]));
    } else {
        const int xs = (x - dx + a.nx) % a.nx, ys = (y - dy + a.ny) % a.ny, zs = (z - dz + a.nz) % a.nz;
        const int src = (zs * a.ny + ys) * a.nx + xs;
        v = static_cast<double>(ST::dec(A[static_cast<size_t>(s * kQ + i) * a.N + src], a.inv_scale)) +
            w * static_cast<double>(a.rho0[s]);
    }
    out[n] = v;
}

template <typename ST>
__global__ void k_set_canonical(Args<typename ST::T> a, const double* __restrict__ in, int s, int i,
                                typename ST::E* __restrict__ A)
{
    using T = typename ST::T;
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
    const int x = n % a.nx, y = (n / a.nx) % a.ny, z = n / (a.nx * a.ny);
    int dx = 0, dy = 0, dz = 0;
    double w = 0;
    for (int k = 0; k < kQ; ++k)
        if (k == i) { dx = CX[k]; dy = CY[k]; dz = CZ[k]; w = wgt<double>(k); }
    // A_i(y) = f_i(y + c_i)
    const int xd = (x + dx + a.nx) % a.nx, yd = (y + dy + a.ny) % a.ny, zd = (z + dz + a.nz) % a.nz;
    const int d = (zd * a.ny + yd) * a.nx + xd;
    const double h = in[d] - w * static_cast<double>(a.rho0[s]);
    A[static_cast<size_t>(s * kQ + i) * a.N + n] = ST::enc(static_cast<T>(h), a.scale);
}

template <typename ST>
__global__ void k_density(Args<typename ST::T> a, int ncomp, const typename ST::E* __restrict__ A,
                          double* __restrict__ rho)
{
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= a.N) return;
    const int x = n % a.nx, y = (n / a.nx) % a.ny, z = n / (a.nx * a.ny);
    const int res = reservoir_of(a, x, y, z);
    const PullIdx q = pull_idx(x, y, z, a.nx, a.ny, a.nz);
    for (int s = 0; s < ncomp; ++s) {
        double acc = 0;
        if (res >= 0) {
            acc = static_cast<double>(a.res_dr[res][s]);
        } else {
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const int src = q.pln[CZ[i] + 1] + q.row[CY[i] + 1] + q.col[CX[i] + 1];
                acc += static_cast<double>(ST::dec(A[static_cast<size_t>(s * kQ + i) * a.N + src], a.inv_scale));
            }
        }
        rho[static_cast<size_t>(s) * a.N + n] = static_cast<double>(a.rho0[s]) + acc;
    }
}

constexpr int kRedThreads = 256;

template <typename ST>
__global__ __launch_bounds__(kRedThreads) void k_moments(Args<typename ST::T> a, int ncomp, int c_ns, double G_s,
                                                         double Gads0, double Gads1, double gG_p,
                                                         const typename ST::E* __restrict__ A,
                                                         const float* __restrict__ ns, const double* __restrict__ rho,
                                                         double* __restrict__ u_out, double* __restrict__ p_out,
                                                         double* __restrict__ partials)
{
    __shared__ double red[5][kRedThreads];
    double acc[5] = {0, 0, 0, 0, 0};
    const double Gads[2] = {Gads0, Gads1};
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < a.N; n += gridDim.x * blockDim.x) {
        const int x = n % a.nx, y = (n / a.nx) % a.ny, z = n / (a.nx * a.ny);
        const int res = reservoir_of(a, x, y, z);
        const PullIdx q = pull_idx(x, y, z, a.nx, a.ny, a.nz);
        // neighbours x + c_i (note: opposite of the pull)
        const int xp = wrap_inc(x, a.nx), xm = wrap_dec(x, a.nx);
        const int yp = wrap_inc(y, a.ny), ym = wrap_dec(y, a.ny);
        const int zp = wrap_inc(z, a.nz), zm = wrap_dec(z, a.nz);
        const int cols[3] = {xm, x, xp}, rows[3] = {ym, y, yp}, plns[3] = {zm, z, zp};
        double rs[2] = {0, 0}, j[2][3] = {{0, 0, 0}, {0, 0, 0}}, rtot = 0;
        for (int s = 0; s < ncomp; ++s) {
            rs[s] = rho[static_cast<size_t>(s) * a.N + n];
            rtot += rs[s];
            if (res < 0) {
#pragma unroll
                for (int i = 0; i < kQ; ++i) {
                    const int src = q.pln[CZ[i] + 1] + q.row[CY[i] + 1] + q.col[CX[i] + 1];
                    const double h = static_cast<double>(ST::dec(A[static_cast<size_t>(s * kQ + i) * a.N + src], a.inv_scale));
                    j[s][0] += CX[i] * h; j[s][1] += CY[i] * h; j[s][2] += CZ[i] * h;
                }
            }
        }
        double m[3] = {0, 0, 0};
        for (int s = 0; s < ncomp; ++s) {
            double gi[3] = {0, 0, 0}, ga[3] = {0, 0, 0};
            const int cn = c_ns == 2 ? s : 0;
#pragma unroll
            for (int i = 1; i < kQ; ++i) {
                const int nb = (plns[CZ[i] + 1] * a.ny + rows[CY[i] + 1]) * a.nx + cols[CX[i] + 1];
                const double wi = wgt<double>(i);
                if (ncomp == 2) {
                    const double r = rho[static_cast<size_t>(1 - s) * a.N + nb];
                    gi[0] += wi * r * CX[i]; gi[1] += wi * r * CY[i]; gi[2] += wi * r * CZ[i];
                }
                const double v = static_cast<double>(ns[static_cast<size_t>(cn) * a.N + nb]);
                ga[0] += wi * v * CX[i]; ga[1] += wi * v * CY[i]; ga[2] += wi * v * CZ[i];
            }
            const double nsx = static_cast<double>(ns[static_cast<size_t>(cn) * a.N + n]);
            for (int d = 0; d < 3; ++d) {
                const double fext = rtot > 0 ? rs[s] / rtot * static_cast<double>(a.F[d]) : 0.0;
                const double ft = -rs[s] * G_s * gi[d] - rs[s] * Gads[s] * ga[d] + fext;
                m[d] += (1.0 - nsx) * (j[s][d] + ft / 2.0);
            }
        }
        double u[3];
        for (int d = 0; d < 3; ++d) u[d] = rtot > 0 ? m[d] / rtot : 0.0;
        if (u_out)
            for (int d = 0; d < 3; ++d) u_out[static_cast<size_t>(d) * a.N + n] = u[d];
        if (p_out) p_out[n] = (rtot + (ncomp == 2 ? gG_p * rs[0] * rs[1] : 0.0)) / 3.0;
        acc[0] += rs[0];
        acc[1] += rs[1];
        for (int d = 0; d < 3; ++d) acc[2 + d] += m[d];
    }
    for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 5) partials[blockIdx.x * 5 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kRedThreads) void k_reduce(const double* __restrict__ partials, int nblocks,
                                                        double* __restrict__ out)
{
    __shared__ double red[5][kRedThreads];
    double acc[5] = {0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblocks; b += kRedThreads)
        for (int k = 0; k < 5; ++k) acc[k] += partials[b * 5 + k];
    for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 5) out[threadIdx.x] = red[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// Launchers.

int storage_bytes(int storage)
{
    switch (storage) {
    case kF64: return 8;
    case kF32: return 4;
    case kF16: return 2;
    case kBF16: return 2;
    default: return 0;
    }
}

template <typename ST, int NC, int CNS, int TY>
static hipError_t step_t(const Problem& p, const Launch& l, const void* A, void* B, const float* ns,
                         hipStream_t st)
{
    using T = typename ST::T;
    using E = typename ST::E;
    Args<T> a = make_args<T>(p);
    a.zchunk = l.zchunk;
    a.ntx = (p.nx + kTileX - 1) / kTileX;
    a.nty = (p.ny + TY - 1) / TY;
    a.nzc = (p.nz + l.zchunk - 1) / l.zchunk;
    const int nblocks = a.ntx * a.nty * a.nzc;
    hipLaunchKernelGGL((k_step<ST, NC, CNS, TY>), dim3(nblocks), dim3(kTileX * TY), 0, st, a,
                       static_cast<const E*>(A), static_cast<E*>(B), ns);
    return hipGetLastError();
}

template <typename ST, int NC, int CNS>
static hipError_t step_ty(const Problem& p, const Launch& l, const void* A, void* B, const float* ns,
                          hipStream_t st)
{
    if (l.tile_y == 4) return step_t<ST, NC, CNS, 4>(p, l, A, B, ns, st);
    if (l.tile_y == 8) return step_t<ST, NC, CNS, 8>(p, l, A, B, ns, st);
    return hipErrorInvalidValue;
}

template <typename ST>
static hipError_t step_st(const Problem& p, const Launch& l, const void* A, void* B, const float* ns,
                          hipStream_t st)
{
    if (p.ncomp == 1) return step_ty<ST, 1, 1>(p, l, A, B, ns, st);
    if (p.c_ns == 1) return step_ty<ST, 2, 1>(p, l, A, B, ns, st);
    return step_ty<ST, 2, 2>(p, l, A, B, ns, st);
}

hipError_t launch_step(const Problem& p, const Launch& l, const void* A, void* B, const float* ns,
                       hipStream_t st)
{
    switch (p.storage) {
    case kF64: return step_st<F64>(p, l, A, B, ns, st);
    case kF32: return step_st<F32>(p, l, A, B, ns, st);
    case kF16: return step_st<F16>(p, l, A, B, ns, st);
    case kBF16: return step_st<BF16>(p, l, A, B, ns, st);
    default: return hipErrorInvalidValue;
    }
}

static unsigned cell_blocks(int64_t N) { return static_cast<unsigned>((N + 255) / 256); }

template <typename F>
static hipError_t by_storage(int storage, F&& f)
{
    switch (storage) {
    case kF64: return f(F64{});
    case kF32: return f(F32{});
    case kF16: return f(F16{});
    case kBF16: return f(BF16{});
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_init(const Problem& p, const double* rho_init, void* A, hipStream_t st)
{
    return by_storage(p.storage, [&](auto tag) {
        using ST = decltype(tag);
        Args<typename ST::T> a = make_args<typename ST::T>(p);
        hipLaunchKernelGGL((k_init<ST>), dim3(cell_blocks(p.N)), dim3(256), 0, st, a, p.ncomp, rho_init,
                           static_cast<typename ST::E*>(A));
        return hipGetLastError();
    });
}

hipError_t launch_canonical(const Problem& p, const void* A, int s, int i, double* out, hipStream_t st)
{
    return by_storage(p.storage, [&](auto tag) {
        using ST = decltype(tag);
        Args<typename ST::T> a = make_args<typename ST::T>(p);
        hipLaunchKernelGGL((k_canonical<ST>), dim3(cell_blocks(p.N)), dim3(256), 0, st, a,
                           static_cast<const typename ST::E*>(A), s, i, out);
        return hipGetLastError();
    });
}

hipError_t launch_set_canonical(const Problem& p, const double* in, int s, int i, void* A, hipStream_t st)
{
    return by_storage(p.storage, [&](auto tag) {
        using ST = decltype(tag);
        Args<typename ST::T> a = make_args<typename ST::T>(p);
        hipLaunchKernelGGL((k_set_canonical<ST>), dim3(cell_blocks(p.N)), dim3(256), 0, st, a, in, s, i,
                           static_cast<typename ST::E*>(A));
        return hipGetLastError();
    });
}

hipError_t launch_density(const Problem& p, const void* A, double* rho, hipStream_t st)
{
    return by_storage(p.storage, [&](auto tag) {
        using ST = decltype(tag);
        Args<typename ST::T> a = make_args<typename ST::T>(p);
        hipLaunchKernelGGL((k_density<ST>), dim3(cell_blocks(p.N)), dim3(256), 0, st, a, p.ncomp,
                           static_cast<const typename ST::E*>(A), rho);
        return hipGetLastError();
    });
}

int moments_max_blocks() { return 1024; }

hipError_t launch_moments(const Problem& p, const void* A, const float* ns, const double* rho, double* u,
                          double* pr, double* partials, int* nblocks, hipStream_t st)
{
    const int nb = static_cast<int>(std::min<int64_t>(moments_max_blocks(), (p.N + kRedThreads - 1) / kRedThreads));
    *nblocks = nb;
    return by_storage(p.storage, [&](auto tag) {
        using ST = decltype(tag);
        Args<typename ST::T> a = make_args<typename ST::T>(p);
        hipLaunchKernelGGL((k_moments<ST>), dim3(nb), dim3(kRedThreads), 0, st, a, p.ncomp, p.c_ns, p.G_s,
                           p.Gads_s[0], p.Gads_s[1], p.g_scale * p.G_inter, static_cast<const typename ST::E*>(A),
                           ns, rho, u, pr, partials);
        return hipGetLastError();
    });
}

hipError_t launch_reduce(const double* partials, int nblocks, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedThreads), 0, st, partials, nblocks, out);
    return hipGetLastError();
}

}  // namespace hm
