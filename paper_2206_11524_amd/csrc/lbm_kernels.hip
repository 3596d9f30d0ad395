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

#include <type_traits>

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
// Buffer resources: raw (stride 0) descriptors whose range check turns any
// access beyond num_records into a zero load / dropped store.  Stores of the
// step are non-temporal (cache-policy bit NT): the next step reads them only
// after the whole domain has streamed through the caches.
using rsrc_t = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf162_t __attribute__((ext_vector_type(2)));
constexpr int kNT = 2;  // cache policy: non-temporal

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), static_cast<short>(0),
                                             static_cast<int>(bytes), 0x00020000);
}

struct F64 {
    using E = double;
    using T = double;
    static __device__ __forceinline__ T dec(E v, T) { return v; }
    static __device__ __forceinline__ E enc(T v, T) { return v; }
    static __device__ __forceinline__ E enc_sr(T v, T, uint32_t) { return v; }  // rounds to nearest
    static __device__ __forceinline__ E bld(rsrc_t r, uint32_t vo, uint32_t so)
    {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    }
    static __device__ __forceinline__ void bst(E v, rsrc_t r, uint32_t vo, uint32_t so)
    {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, vo, so, kNT);
    }
};
struct F32 {
    using E = float;
    using T = float;
    static __device__ __forceinline__ T dec(E v, T) { return v; }
    static __device__ __forceinline__ E enc(T v, T) { return v; }
    static __device__ __forceinline__ E enc_sr(T v, T, uint32_t) { return v; }  // rounds to nearest
    static __device__ __forceinline__ E bld(rsrc_t r, uint32_t vo, uint32_t so)
    {
        return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
    }
    static __device__ __forceinline__ void bst(E v, rsrc_t r, uint32_t vo, uint32_t so)
    {
        __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, vo, so, kNT);
    }
};
struct Half16 {
    static __device__ __forceinline__ uint16_t bld(rsrc_t r, uint32_t vo, uint32_t so)
    {
        return __builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0);
    }
    static __device__ __forceinline__ void bst(uint16_t v, rsrc_t r, uint32_t vo, uint32_t so)
    {
        __builtin_amdgcn_raw_buffer_store_b16(v, r, vo, so, kNT);
    }
};
struct F16 : Half16 {
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
    // Stochastic rounding with 16 random bits r16 (v_cvt_sr_f16_f32): the
    // instruction reads its random operand as a binary fraction from the top
    // bit down and rounds the magnitude up with probability equal to the
    // value's fraction of the binary16 spacing, subnormals included (checked
    // on the device: up only for bit 31 at half a spacing, frequencies equal
    // to the fraction, exact values unchanged, inf and NaN kept).  r16 goes to
    // the top half, so the probability is resolved to 2^-16.
    static __device__ __forceinline__ E enc_sr(T v, T scale, uint32_t r16)
    {
        half2_t h = {0, 0};
        h = __builtin_amdgcn_cvt_sr_f16_f32(h, v * scale, r16 << 16, false);
        return __builtin_bit_cast(uint16_t, h[0]);
    }
};
struct BF16 : Half16 {
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
    // Stochastic rounding with 16 random bits (v_cvt_sr_bf16_f32, the same
    // convention as the binary16 instruction).
    static __device__ __forceinline__ E enc_sr(T v, T scale, uint32_t r16)
    {
        bf162_t h = {0, 0};
        h = __builtin_amdgcn_cvt_sr_bf16_f32(h, v * scale, r16 << 16, false);
        return __builtin_bit_cast(uint16_t, h[0]);
    }
};

// MurmurHash3's 32-bit finaliser (Appleby): a bijective avalanche mixer; the
// random bits of the stochastic rounding are fmix32 of a counter built from
// cell, component, direction and time step.
__device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}
constexpr uint32_t kGolden = 0x9e3779b9u;

// Marsaglia's xorshift32 step (shifts 13, 17, 5): the following random words
// of one cell, after fmix32 has seeded them.
__device__ __forceinline__ uint32_t xorshift32(uint32_t x)
{
    x ^= x << 13;
    x ^= x >> 17;
    x ^= x << 5;
    return x;
}

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
    T guo[2];    // 1 - 1/(2 tau): weight of the Guo forcing term (GS-WBS)
    int sr;      // stochastic rounding of stored values
    uint32_t t;  // time step of the state read by the launch (single-domain launches)
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
        a.guo[s] = static_cast<T>(1.0 - 0.5 / p.tau[s]);
        a.Gads_s[s] = static_cast<T>(p.Gads_s[s]);
        a.rho0[s] = static_cast<T>(p.rho0[s]);
    }
    a.G_s = static_cast<T>(p.G_s);
    for (int d = 0; d < 3; ++d) a.F[d] = static_cast<T>(p.F[d]);
    a.scale = static_cast<T>(p.scale);
    a.inv_scale = static_cast<T>(1.0 / p.scale);
    a.sr = p.stochastic;
    a.t = 0;
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

// The same search for the step kernel, returning the shifted density of
// component s in that reservoir.  The loop runs over the slots with
// compile-time indices and s is the same for the whole wave, so every
// parameter is read with scalar loads (a per-lane indexed load would be a
// vector memory load, and waiting for it would wait for every load issued
// before it).
template <typename T>
__device__ __forceinline__ bool reservoir_dr(const Args<T>& a, int s, int x, int y, int z, T& dr)
{
    bool in = false;
    dr = T(0);
#pragma unroll
    for (int r = 0; r < kMaxRes; ++r) {
        if (r < a.n_res) {
            const int c = a.res_axis[r] == 0 ? x : (a.res_axis[r] == 1 ? y : z);
            const bool hit = !in && c >= a.res_lo[r] && c < a.res_hi[r];
            dr = hit ? (s == 0 ? a.res_dr[r][0] : a.res_dr[r][1]) : dr;
            in = in || hit;
        }
    }
    return in;
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

// Fused step kernel.
//
// Addressing: the pull source of direction i at cell (x, y, z) is the cell
// (x - cx, y - cy, z - cz).  Its plane part is uniform across the block, so it
// is folded into a per-direction base pointer computed on the scalar unit; the
// in-plane part takes one of nine values per thread, computed once before the
// z sweep.  Loads are therefore "uniform base + 32-bit lane offset".
template <typename E>
__device__ __forceinline__ E ld_off(const E* base, uint32_t byte_off)
{
    return *reinterpret_cast<const E*>(reinterpret_cast<const char*>(base) + byte_off);
}

template <typename E>
__device__ __forceinline__ void st_off(E* base, uint32_t byte_off, E v)
{
    *reinterpret_cast<E*>(reinterpret_cast<char*>(base) + byte_off) = v;
}

// In-plane byte offsets of the nine (x - cx, y - cy) sources of a cell.
struct PlaneOffs {
    uint32_t o[3][3];  // [cy + 1][cx + 1]
};

template <typename E>
__device__ __forceinline__ PlaneOffs plane_offs(int x, int y, int nx, int ny)
{
    const int xs[3] = {x == nx - 1 ? 0 : x + 1, x, x == 0 ? nx - 1 : x - 1};  // x - c, c = -1, 0, 1
    const int ys[3] = {y == ny - 1 ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
    PlaneOffs q;
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) q.o[b][a] = static_cast<uint32_t>((ys[b] * nx + xs[a]) * static_cast<int>(sizeof(E)));
    return q;
}

// Pull the shifted pre-collision populations of one cell and component.
// r covers the 19 direction arrays of component s; soff[c + 1] is the byte
// offset of the source plane z - c; q holds the in-plane byte offsets.
template <typename ST, typename T>
__device__ __forceinline__ void pull(rsrc_t r, uint32_t dir_bytes, const uint32_t soff[3], const PlaneOffs& q,
                                     T inv_scale, T h[kQ])
{
#pragma unroll
    for (int i = 0; i < kQ; ++i)
        h[i] = ST::dec(ST::bld(r, q.o[CY[i] + 1][CX[i] + 1], soff[CZ[i] + 1] + static_cast<uint32_t>(i) * dir_bytes),
                       inv_scale);
}

// The same loads without decoding: the raw values can stay in flight while
// other work runs, and are decoded where they are consumed.
template <typename ST>
__device__ __forceinline__ void pull_raw(rsrc_t r, uint32_t dir_bytes, const uint32_t soff[3], const PlaneOffs& q,
                                         typename ST::E e[kQ])
{
#pragma unroll
    for (int i = 0; i < kQ; ++i)
        e[i] = ST::bld(r, q.o[CY[i] + 1][CX[i] + 1], soff[CZ[i] + 1] + static_cast<uint32_t>(i) * dir_bytes);
}

template <typename T>
__device__ __forceinline__ T sum19(const T h[kQ])
{
    T acc = h[0];
#pragma unroll
    for (int i = 1; i <= 9; ++i) acc += h[i] + h[i + 9];
    return acc;
}

// sum_i sign(c_ia) v_i over the directions with c_ia != 0, paired i / i+9
template <typename T, int AX>
__device__ __forceinline__ T first_moment(const T h[kQ])
{
    T acc = T(0);
#pragma unroll
    for (int i = 1; i <= 9; ++i) {
        const int c = AX == 0 ? CX[i] : (AX == 1 ? CY[i] : CZ[i]);
        if (c) acc += c > 0 ? h[i] - h[i + 9] : h[i + 9] - h[i];
    }
    return acc;
}

// Neighbour stencil sum_i w_i phi(x + c_i) c_i read from an LDS plane triple.
template <typename T, typename V, int LW>
__device__ __forceinline__ void stencil(const V* pm, const V* p0, const V* pp, int me, T g[3])
{
    // group by weight: axis neighbours (1/18) and diagonals (1/36)
    T ax[3] = {0, 0, 0}, dg[3] = {0, 0, 0};
#pragma unroll
    for (int i = 1; i < kQ; ++i) {
        const V* pl = CZ[i] == 0 ? p0 : (CZ[i] > 0 ? pp : pm);
        const T v = static_cast<T>(pl[me + CY[i] * LW + CX[i]]);
        const bool axis = (CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i]) == 1;
        T* acc = axis ? ax : dg;
        if (CX[i]) acc[0] += CX[i] > 0 ? v : -v;
        if (CY[i]) acc[1] += CY[i] > 0 ? v : -v;
        if (CZ[i]) acc[2] += CZ[i] > 0 ? v : -v;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) g[d] = ax[d] * (T(1) / T(18)) + dg[d] * (T(1) / T(36));
}

// 1/x: correctly rounded in FP64; in FP32 the hardware reciprocal (within
// one unit in the last place), one instruction instead of a division
template <typename T>
__device__ __forceinline__ T recip(T x)
{
    if constexpr (sizeof(T) == 4) return __builtin_amdgcn_rcpf(x);
    else return T(1) / x;
}

// Per-cell physics shared by the step kernels: every kernel evaluates the
// same expressions, so the result of a cell does not depend on which kernel
// or launch shape updated it.

// Equilibrium velocity of component s at one cell, Eq. (SC_u_eq): the common
// velocity sum_c (j_c / tau_c) / sum_c (rho_c / tau_c) plus tau_s F_tot,s /
// rho_s, with F_tot,s the sum of Eqs. (SC_F_inter), (SC_F_ads) and
// (SC_F_ext); no force shift for an absent component.  rho_m/0/p point at the
// LDS density planes z-1, z, z+1 ([NC][LP]), ns_m/0/p at the n_s planes
// ([CNS][LP]); me is the cell's LDS index and jc[c] the first moment of
// component c at the cell.  Also returns the own density and n_s.
template <typename T, int NC, int CNS, int LW, int LP>
__device__ __forceinline__ void cell_velocity(const Args<T>& a, int s, int me, const T* rho_m, const T* rho_0,
                                              const T* rho_p, const float* ns_m, const float* ns_0,
                                              const float* ns_p, const T (&jc)[NC][3], T ueq[3], T& rho_own, T& n)
{
    T rho = 0, den = 0, num[3] = {0, 0, 0};
    rho_own = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const T rc = rho_0[c * LP + me];
        if (c == s) rho_own = rc;
        rho += rc;
        den += rc * a.inv_tau[c];
#pragma unroll
        for (int d = 0; d < 3; ++d) num[d] += jc[c][d] * a.inv_tau[c];
    }
    const T inv_den = den > T(0) ? recip(den) : T(0);
    const T inv_rho = rho > T(0) ? recip(rho) : T(0);
    const int cn = CNS == 2 ? s : 0;
    T ga[3];
    stencil<T, float, LW>(ns_m + cn * LP, ns_0 + cn * LP, ns_p + cn * LP, me, ga);
    T gi[3] = {0, 0, 0};
    if constexpr (NC == 2) stencil<T, T, LW>(rho_m + (1 - s) * LP, rho_0 + (1 - s) * LP, rho_p + (1 - s) * LP, me, gi);
    const bool present = rho_own > T(0);
    const T tau_s = a.tau[s], Gads = a.Gads_s[s];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T acc = -a.G_s * gi[d] - Gads * ga[d] + a.F[d] * inv_rho;
        ueq[d] = num[d] * inv_den + (present ? tau_s * acc : T(0));
    }
    n = static_cast<T>(ns_0[cn * LP + me]);
}

// The GS-WBS of Eq. (GS-WBS) takes its equilibrium at u_macro of
// Eq. (HMCSC_u_macro), common to the components: sum_c (1 - n_c)(j_c +
// F_tot,c / 2) / rho.  That needs the total force of every component at the
// cell (both cohesion stencils); returns u_macro, the own total force, the own
// density and n_s.
template <typename T, int NC, int CNS, int LW, int LP>
__device__ __forceinline__ void cell_velocity_guo(const Args<T>& a, int s, int me, const T* rho_m, const T* rho_0,
                                                  const T* rho_p, const float* ns_m, const float* ns_0,
                                                  const float* ns_p, const T (&jc)[NC][3], T um[3], T fo[3],
                                                  T& rho_own, T& n_own)
{
    T rc[NC], rho = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        rc[c] = rho_0[c * LP + me];
        rho += rc[c];
    }
    const T inv_rho = rho > T(0) ? recip(rho) : T(0);
    T m[3] = {0, 0, 0};
    T ga[3];
    if constexpr (CNS == 1) stencil<T, float, LW>(ns_m, ns_0, ns_p, me, ga);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const int cn = CNS == 2 ? c : 0;
        if constexpr (CNS == 2) stencil<T, float, LW>(ns_m + cn * LP, ns_0 + cn * LP, ns_p + cn * LP, me, ga);
        T gi[3] = {0, 0, 0};
        if constexpr (NC == 2)
            stencil<T, T, LW>(rho_m + (1 - c) * LP, rho_0 + (1 - c) * LP, rho_p + (1 - c) * LP, me, gi);
        const T nc = static_cast<T>(ns_0[cn * LP + me]);
        T F[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            F[d] = rc[c] * (-a.G_s * gi[d] - a.Gads_s[c] * ga[d] + a.F[d] * inv_rho);
            m[d] += (T(1) - nc) * (jc[c][d] + T(0.5) * F[d]);
        }
        if (c == s) {
#pragma unroll
            for (int d = 0; d < 3; ++d) fo[d] = F[d];
            rho_own = rc[c];
            n_own = nc;
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) um[d] = m[d] * inv_rho;
}

// Force-shifted BGK collision blended with partial bounce-back, Eq. (LGS), in
// the shifted variables: post_i = (1-n)(h_i - (h_i - h^eq_i)/tau_s) + n h_ibar
// with h^eq from Eq. (Maxwell) at u_eq (the w_i rho0 shift cancels because
// w_ibar = w_i).  relax_coef gathers the per-cell factors, relax_dir gives the
// results of one direction pair (i, i+9), relax_rest that of direction 0.
template <typename T>
struct RelaxCoef {
    T ca, n;                  // weights of h_i and h_ibar
    T K0[3], K1[3], K2[3];    // weight of h^eq_i: K0 + K1 c.u + K2 (c.u)^2 per weight class
    T u[3];
};

template <typename T>
__device__ __forceinline__ RelaxCoef<T> relax_coef(const Args<T>& a, int s, T rho_own, const T ueq[3], T n)
{
    RelaxCoef<T> k;
    const T uu = ueq[0] * ueq[0] + ueq[1] * ueq[1] + ueq[2] * ueq[2];
    const T omn = T(1) - n;
    const T cb = omn * a.inv_tau[s];  // weight of h^eq
    k.ca = omn - cb;                  // weight of h
    k.n = n;
    const T base0 = (rho_own - a.rho0[s]) - T(1.5) * rho_own * uu;
    const T r3 = T(3) * rho_own, r45 = T(4.5) * rho_own;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const T wk = cb * (c == 0 ? T(1) / T(3) : (c == 1 ? T(1) / T(18) : T(1) / T(36)));
        k.K0[c] = wk * base0;
        k.K1[c] = wk * r3;
        k.K2[c] = wk * r45;
        k.u[c] = ueq[c];
    }
    return k;
}

template <typename T>
__device__ __forceinline__ T relax_rest(const RelaxCoef<T>& k, T h0)
{
    return k.ca * h0 + k.n * h0 + k.K0[0];
}

// i in 1..9: hi = h_i, ho = h_{i+9}
template <typename T>
__device__ __forceinline__ void relax_dir(const RelaxCoef<T>& k, int i, T hi, T ho, T& post_i, T& post_o)
{
    const int c = (CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i]) == 1 ? 1 : 2;
    T cu = T(0);
    if (CX[i]) cu += CX[i] > 0 ? k.u[0] : -k.u[0];
    if (CY[i]) cu += CY[i] > 0 ? k.u[1] : -k.u[1];
    if (CZ[i]) cu += CZ[i] > 0 ? k.u[2] : -k.u[2];
    const T t = k.K2[c] * (cu * cu) + k.K0[c];
    const T e = k.K1[c] * cu;
    post_i = k.ca * hi + (k.n * ho + (t + e));
    post_o = k.ca * ho + (k.n * hi + (t - e));
}

// The forcing term of Guo, Zheng and Shi (2002), weighted by (1 - n_s) as in
// Eq. (GS-WBS): F_i = A w_i [3 (c_i - u).F + 9 (c_i.u)(c_i.F)] with
// A = (1 - n)(1 - 1/(2 tau)).  For a pair (i, ibar) the part even in c_i,
// A w (9 cu cF - 3 u.F), adds to both, the odd part A w 3 cF with opposite
// signs, as in relax_dir.
template <typename T>
struct GuoCoef {
    T gw[3];   // A w per weight class
    T f[3];    // F_tot of the component
    T uF;
};

template <typename T>
__device__ __forceinline__ GuoCoef<T> guo_coef(const Args<T>& a, int s, T n, const T F[3], const T u[3])
{
    GuoCoef<T> g;
    const T A = (T(1) - n) * a.guo[s];
#pragma unroll
    for (int c = 0; c < 3; ++c) g.gw[c] = A * (c == 0 ? T(1) / T(3) : (c == 1 ? T(1) / T(18) : T(1) / T(36)));
#pragma unroll
    for (int d = 0; d < 3; ++d) g.f[d] = F[d];
    g.uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    return g;
}

template <typename T>
__device__ __forceinline__ T relax_rest_guo(const RelaxCoef<T>& k, const GuoCoef<T>& g, T h0)
{
    return k.ca * h0 + k.n * h0 + (k.K0[0] + g.gw[0] * (T(-3) * g.uF));
}

template <typename T>
__device__ __forceinline__ void relax_dir_guo(const RelaxCoef<T>& k, const GuoCoef<T>& g, int i, T hi, T ho,
                                              T& post_i, T& post_o)
{
    const int c = (CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i]) == 1 ? 1 : 2;
    T cu = T(0), cF = T(0);
    if (CX[i]) { cu += CX[i] > 0 ? k.u[0] : -k.u[0]; cF += CX[i] > 0 ? g.f[0] : -g.f[0]; }
    if (CY[i]) { cu += CY[i] > 0 ? k.u[1] : -k.u[1]; cF += CY[i] > 0 ? g.f[1] : -g.f[1]; }
    if (CZ[i]) { cu += CZ[i] > 0 ? k.u[2] : -k.u[2]; cF += CZ[i] > 0 ? g.f[2] : -g.f[2]; }
    const T t = k.K2[c] * (cu * cu) + k.K0[c] + g.gw[c] * (T(9) * (cu * cF) - T(3) * g.uF);
    const T e = k.K1[c] * cu + g.gw[c] * (T(3) * cF);
    post_i = k.ca * hi + (k.n * ho + (t + e));
    post_o = k.ca * ho + (k.n * hi + (t - e));
}

// One thread per (cell, component): a block of NC*TX*TY threads owns a TX x TY
// column of cells; threads [s*TX*TY, (s+1)*TX*TY) handle component s.  The two
// components of a cell meet only through LDS (densities and first moments),
// which halves the registers per thread and doubles the waves per CU.
//
// LDS holds four density / n_s plane slots (plane p in slot p mod 4) and three
// first-moment slots (p mod 3), so one barrier per plane suffices: a wave that
// runs ahead into staging plane z+2 writes slots that no wave still colliding
// plane z reads, and every wave has left the collision of plane z-1 before the
// barrier that precedes the collision of plane z.
template <typename ST, int NC, int CNS, int TX, int TY>
struct TileShared {
    using T = typename ST::T;
    static constexpr int LW = TX + 2;
    static constexpr int LP = LW * (TY + 2);
    static constexpr int NTC = TX * TY;
    static constexpr int NT = NC * NTC;
    // Where the tile fits the 160 KB of LDS with it: the populations of the
    // plane staged last wait here (private to each thread) until it is
    // collided, which frees the registers that keep the next plane's loads
    // in flight (the three-plane sweep of step_tile)
    static constexpr size_t kBase = sizeof(T) * (4 * NC * LP + 3 * NC * 3 * NTC) + sizeof(float) * 4 * CNS * LP;
    static constexpr bool kPipe = kBase + sizeof(T) * kQ * NT <= 160 * 1024;
    T rho[4][NC][LP];
    float ns[4][CNS][LP];
    T j[3][NC][3][NTC];
    T hs[kPipe ? kQ : 1][kPipe ? NT : 1];
};

// The sweep of one tile column (logical tile index L of the domain described
// by a).  Shared by the single-domain and the batched kernels.
template <typename ST, int NC, int CNS, int TX, int TY, int FS, bool ONE = false>
__device__ __forceinline__ void step_tile(const Args<typename ST::T>& a, const typename ST::E* __restrict__ A,
                                          typename ST::E* __restrict__ B, const float* __restrict__ ns, int L,
                                          uint32_t t, TileShared<ST, NC, CNS, TX, TY>& sh)
{
    using T = typename ST::T;
    using E = typename ST::E;
    constexpr int LW = TX + 2;
    constexpr int LP = LW * (TY + 2);
    constexpr int NTC = TX * TY;  // threads per component
    constexpr int NT = NC * NTC;
    constexpr int NSMAX = (LP + NT - 1) / NT;  // n_s cells staged per thread and plane
    auto& s_rho = sh.rho;
    auto& s_ns = sh.ns;
    auto& s_j = sh.j;

    const int tx = L % a.ntx;
    const int ty = (L / a.ntx) % a.nty;
    const int tz = L / (a.ntx * a.nty);
    const int x0 = tx * TX, y0 = ty * TY;
    const int zs = tz * a.zchunk;
    const int ze = min(zs + a.zchunk, a.nz);
    const int TXe = min(TX, a.nx - x0);
    const int TYe = min(TY, a.ny - y0);
    const int plane = a.nx * a.ny;

    // component of this thread; NTC is a multiple of 64, so it is the same
    // for every lane of a wave: saying so keeps the buffer descriptors and
    // everything derived from s in scalar registers (otherwise each load
    // becomes a loop over the distinct descriptor values of the wave)
    const int s = NC == 1 ? 0 : __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / NTC);
    static_assert(NTC % 64 == 0, "a wave must not straddle two components");
    const int tl = static_cast<int>(threadIdx.x) - s * NTC;
    const int lx = tl % TX;
    const int ly = tl / TX;
    const bool act = lx < TXe && ly < TYe;
    const int x = x0 + min(lx, TXe - 1);
    const int y = y0 + min(ly, TYe - 1);
    // LDS cell and first-moment slot of the (clamped) own cell: a lane beyond
    // a ragged tile edge duplicates the last active lane of its row/column
    const int me = (y - y0 + 1) * LW + (x - x0 + 1);
    const int tj = (y - y0) * TX + (x - x0);
    const PlaneOffs qme = plane_offs<E>(x, y, a.nx, a.ny);
    const uint32_t own = static_cast<uint32_t>((y * a.nx + x) * static_cast<int>(sizeof(E)));

    // ring cell of this thread (if any): top row, bottom row, left, right column
    const int ring_n = 2 * (TXe + 2) + 2 * TYe;
    const bool ring = NC == 2 && tl < ring_n;  // only the cohesion stencil reads ring densities
    int rlx, rly;
    {
        const int r = min(tl, ring_n - 1);
        if (r < TXe + 2) { rlx = r - 1; rly = -1; }
        else if (r < 2 * (TXe + 2)) { rlx = r - (TXe + 2) - 1; rly = TYe; }
        else if (r < 2 * (TXe + 2) + TYe) { rlx = -1; rly = r - 2 * (TXe + 2); }
        else { rlx = TXe; rly = r - 2 * (TXe + 2) - TYe; }
    }
    const int rx = ((x0 + rlx) % a.nx + a.nx) % a.nx;
    const int ry = ((y0 + rly) % a.ny + a.ny) % a.ny;
    const int rme = (rly + 1) * LW + (rlx + 1);
    const PlaneOffs qring = plane_offs<E>(rx, ry, a.nx, a.ny);

    // n_s cells staged by this thread: LDS index and in-plane offset
    const int nsw = TXe + 2, nsh = TYe + 2;
    int ns_lds[NSMAX], ns_off[NSMAX];
#pragma unroll
    for (int k = 0; k < NSMAX; ++k) {
        const int c = static_cast<int>(threadIdx.x) + k * NT;
        if (c < nsw * nsh) {
            const int llx = c % nsw - 1, lly = c / nsw - 1;
            const int gx = ((x0 + llx) % a.nx + a.nx) % a.nx;
            const int gy = ((y0 + lly) % a.ny + a.ny) % a.ny;
            ns_lds[k] = (lly + 1) * LW + llx + 1;
            ns_off[k] = gy * a.nx + gx;
        } else {
            ns_lds[k] = -1;
            ns_off[k] = 0;
        }
    }

    auto wrapz = [&](int p) { return p < 0 ? p + a.nz : (p >= a.nz ? p - a.nz : p); };
    const uint32_t t_key = fmix32(t ^ kGolden);  // stochastic rounding: time part of the counter

    const uint32_t dir_bytes = static_cast<uint32_t>(a.N * static_cast<int>(sizeof(E)));
    const uint32_t plane_bytes = static_cast<uint32_t>(plane * static_cast<int>(sizeof(E)));
    // one buffer descriptor per component spans its 19 direction arrays
    const uint32_t comp_bytes = static_cast<uint32_t>(kQ) * dir_bytes;
    const rsrc_t ra = make_rsrc(A + static_cast<size_t>(s * kQ) * static_cast<size_t>(a.N), comp_bytes);
    const rsrc_t rb = make_rsrc(B + static_cast<size_t>(s * kQ) * static_cast<size_t>(a.N), comp_bytes);

    auto pull_plane = [&](int p, const PlaneOffs& q, T h[kQ]) {
        const uint32_t so[3] = {static_cast<uint32_t>(wrapz(p + 1)) * plane_bytes,  // c_z = -1
                                static_cast<uint32_t>(p) * plane_bytes,
                                static_cast<uint32_t>(wrapz(p - 1)) * plane_bytes};  // c_z = +1
        pull<ST, T>(ra, dir_bytes, so, q, a.inv_scale, h);
    };
    // A select per value rather than a per-lane branch: in divergent control
    // flow a branch makes the compiler merge the two versions of all 19
    // values through copies, doubling the registers they hold.  The selects
    // are skipped as a whole when no lane of the wave is in a reservoir (the
    // common case; a branch taken by the whole wave).
    auto reservoir_override = [&](int cx, int cy, int cz, T h[kQ]) {
        T dr;
        const bool in = reservoir_dr(a, s, cx, cy, cz, dr);
        if (__builtin_amdgcn_ballot_w64(in) != 0) {
#pragma unroll
            for (int i = 0; i < kQ; ++i) h[i] = in ? wgt<T>(i) * dr : h[i];
        }
    };

    // Stage plane p into LDS slot `slot`: densities of the own cell and of
    // the ring cell, first moments of the own cell (slot js, none if js < 0),
    // n_s; the own cell's populations stay in h for the collision.
    auto stage_plane = [&](int p, int slot, int js, T h[kQ]) {
        // issue the own and the ring loads before either is consumed, so a
        // ring lane waits for one memory round trip per plane, not two
        T hr[kQ];
        if (act) pull_plane(p, qme, h);
        if (ring) pull_plane(p, qring, hr);
        if (act) {
            reservoir_override(x, y, p, h);
            s_rho[slot][s][me] = a.rho0[s] + sum19(h);
            if (NC == 2 && js >= 0) {
                s_j[js][s][0][tj] = first_moment<T, 0>(h);
                s_j[js][s][1][tj] = first_moment<T, 1>(h);
                s_j[js][s][2][tj] = first_moment<T, 2>(h);
            }
        }
        if (ring) {
            reservoir_override(rx, ry, p, hr);
            s_rho[slot][s][rme] = a.rho0[s] + sum19(hr);
        }
        const float* nsp = ns + static_cast<size_t>(p) * plane;
#pragma unroll
        for (int k = 0; k < NSMAX; ++k)
            if (ns_lds[k] >= 0)
#pragma unroll
                for (int c = 0; c < CNS; ++c) s_ns[slot][c][ns_lds[k]] = nsp[static_cast<size_t>(c) * a.N + ns_off[k]];
    };

    // Collision of plane z of this thread's component from h (pre-collision,
    // shifted) and the LDS slots of planes z-1, z, z+1.
    auto collide = [&](int z, int sm, int s0, int sp, int js, const T h[kQ], bool guard) {
        if (guard && !act) return;
        T jc[NC][3];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            if constexpr (NC == 1) {
                jc[c][0] = first_moment<T, 0>(h);
                jc[c][1] = first_moment<T, 1>(h);
                jc[c][2] = first_moment<T, 2>(h);
            } else {
#pragma unroll
                for (int d = 0; d < 3; ++d) jc[c][d] = s_j[js][c][d][tj];
            }
        }
        T ueq[3], rho_own, n, fo[3];
        if constexpr (FS == kForcingGuo)
            cell_velocity_guo<T, NC, CNS, LW, LP>(a, s, me, &s_rho[sm][0][0], &s_rho[s0][0][0], &s_rho[sp][0][0],
                                                  &s_ns[sm][0][0], &s_ns[s0][0][0], &s_ns[sp][0][0], jc, ueq, fo,
                                                  rho_own, n);
        else
            cell_velocity<T, NC, CNS, LW, LP>(a, s, me, &s_rho[sm][0][0], &s_rho[s0][0][0], &s_rho[sp][0][0],
                                              &s_ns[sm][0][0], &s_ns[s0][0][0], &s_ns[sp][0][0], jc, ueq, rho_own, n);
        const uint32_t zo = static_cast<uint32_t>(z) * plane_bytes;
        const RelaxCoef<T> k = relax_coef<T>(a, s, rho_own, ueq, n);
        GuoCoef<T> g{};
        if constexpr (FS == kForcingGuo) g = guo_coef<T>(a, s, n, fo, ueq);
        auto rest = [&]() {
            if constexpr (FS == kForcingGuo) return relax_rest_guo(k, g, h[0]);
            else return relax_rest(k, h[0]);
        };
        auto pair = [&](int i, T& pi, T& po) {
            if constexpr (FS == kForcingGuo) relax_dir_guo(k, g, i, h[i], h[i + 9], pi, po);
            else relax_dir(k, i, h[i], h[i + 9], pi, po);
        };
        if (a.sr) {
            // counter: (cell, component) mixed with the time step, then the direction
            // 32 random bits per direction pair (i, i+9), 16 for each value:
            // fmix32 of (cell, component, time), then xorshift32 steps
            const uint32_t cell = static_cast<uint32_t>(z * plane + y * a.nx + x);
            uint32_t r = fmix32(t_key ^ (2u * cell + static_cast<uint32_t>(s))) | 1u;  // nonzero state
            ST::bst(ST::enc_sr(rest(), a.scale, r >> 16), rb, own, zo);
#pragma unroll
            for (int i = 1; i <= 9; ++i) {
                T pi, po;
                pair(i, pi, po);
                r = xorshift32(r);
                ST::bst(ST::enc_sr(pi, a.scale, r & 0xffffu), rb, own, zo + static_cast<uint32_t>(i) * dir_bytes);
                ST::bst(ST::enc_sr(po, a.scale, r >> 16), rb, own, zo + static_cast<uint32_t>(i + 9) * dir_bytes);
            }
        } else {
            ST::bst(ST::enc(rest(), a.scale), rb, own, zo);
#pragma unroll
            for (int i = 1; i <= 9; ++i) {
                T pi, po;
                pair(i, pi, po);
                ST::bst(ST::enc(pi, a.scale), rb, own, zo + static_cast<uint32_t>(i) * dir_bytes);
                ST::bst(ST::enc(po, a.scale), rb, own, zo + static_cast<uint32_t>(i + 9) * dir_bytes);
            }
        }
    };

    // plane p (zs-1 <= p <= ze) uses density slot (p - zs + 1) mod 4 and
    // first-moment slot (p - zs) mod 3
    auto rslot = [&](int p) { return (p - zs + 1) & 3; };
    auto jslot = [&](int p) { return (p - zs) % 3; };

    if constexpr (TileShared<ST, NC, CNS, TX, TY>::kPipe) {
        // Three planes at a time: plane z is collided from registers, plane
        // z+1 waits in LDS (hs), and the own loads of plane z+2 are in flight
        // over the barrier and the collision of plane z.
        //
        // The compiler counts outstanding memory operations per control-flow
        // path, and after a branch that may have skipped some it has to wait
        // as if they had been issued last; a load or store under a per-lane
        // condition would therefore make every later wait drain the loads
        // kept in flight.  So nothing here touches memory conditionally:
        // lanes beyond a ragged tile edge duplicate an active lane (same
        // cell, same LDS slots, identical values written twice), lanes
        // without a ring cell load at offsets past the buffer's range
        // (dropped by the range check), and lanes without an n_s cell
        // duplicate cell 0 of the staging list.
        constexpr int NT_ = TileShared<ST, NC, CNS, TX, TY>::NT;
        constexpr uint32_t kOff = 0x80000000u;  // beyond any buffer of a single component below 2 GiB
        T* hs = &sh.hs[0][0] + threadIdx.x;
        PlaneOffs qr = qring;
        if (!ring)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int c = 0; c < 3; ++c) qr.o[b][c] |= kOff;
        // list cell 0 is the corner (x0 - 1, y0 - 1), LDS index 0
        const int ns_off0 = (((y0 - 1) % a.ny + a.ny) % a.ny) * a.nx + ((x0 - 1) % a.nx + a.nx) % a.nx;
        int nl[NSMAX], no[NSMAX];
#pragma unroll
        for (int k = 0; k < NSMAX; ++k) {
            nl[k] = ns_lds[k] >= 0 ? ns_lds[k] : 0;
            no[k] = ns_lds[k] >= 0 ? ns_off[k] : ns_off0;
        }
        auto issue = [&](int p, const PlaneOffs& q, E e[kQ]) {
            const uint32_t so[3] = {static_cast<uint32_t>(wrapz(p + 1)) * plane_bytes,
                                    static_cast<uint32_t>(p) * plane_bytes,
                                    static_cast<uint32_t>(wrapz(p - 1)) * plane_bytes};
            pull_raw<ST>(ra, dir_bytes, so, q, e);
        };
        if constexpr (ONE) {
            // One cell deep (the instance launched for nz = 1): planes z - 1,
            // z and z + 1 are all plane 0, so it is staged once and collided
            // against itself (one memory round trip per step instead of the
            // sweep's three; the three slots the sweep would fill hold the
            // same values).  A kernel of its own: as a branch in the 3-D
            // kernels it changed their register allocation.
            const int slot = rslot(0), js = jslot(0);
            E r1[kQ];
            E r2[NC == 2 ? kQ : 1];
            issue(0, qme, r1);
            if constexpr (NC == 2) issue(0, qr, r2);
            float nsv[NSMAX][CNS];
#pragma unroll
            for (int k = 0; k < NSMAX; ++k)
#pragma unroll
                for (int c = 0; c < CNS; ++c) nsv[k][c] = ns[static_cast<size_t>(c) * a.N + no[k]];
            T h[kQ];
#pragma unroll
            for (int i = 0; i < kQ; ++i) h[i] = ST::dec(r1[i], a.inv_scale);
            reservoir_override(x, y, 0, h);
            s_rho[slot][s][me] = a.rho0[s] + sum19(h);
            if constexpr (NC == 2) {
                s_j[js][s][0][tj] = first_moment<T, 0>(h);
                s_j[js][s][1][tj] = first_moment<T, 1>(h);
                s_j[js][s][2][tj] = first_moment<T, 2>(h);
                if (ring) {
                    T hr[kQ];
#pragma unroll
                    for (int i = 0; i < kQ; ++i) hr[i] = ST::dec(r2[i], a.inv_scale);
                    reservoir_override(rx, ry, 0, hr);
                    s_rho[slot][s][rme] = a.rho0[s] + sum19(hr);
                }
            }
#pragma unroll
            for (int k = 0; k < NSMAX; ++k)
#pragma unroll
                for (int c = 0; c < CNS; ++c) s_ns[slot][c][nl[k]] = nsv[k][c];
            __syncthreads();
            collide(0, slot, slot, slot, js, h, false);
            return;
        }
        if constexpr (sizeof(E) != 2) {
            E rr[kQ];  // own populations of the next plane to stage, raw
            E er[kQ];  // ring populations of the plane being staged, raw
            // Stage plane p, whose own loads are in rr: ring loads and n_s are
            // issued first; the own values give the density and first moments
            // and go to hs, whose previous content (the plane before) moves to
            // hz; then the own loads of plane pn are issued, and only after them
            // the ring values are consumed, so a wait for the ring does not wait
            // for plane pn.
            auto stage_pipe = [&](int p, int slot, int js, int pn, T hz[kQ]) {
                if constexpr (NC == 2) issue(p, qr, er);
                const float* nsp = ns + static_cast<size_t>(p) * plane;
                float nsv[NSMAX][CNS];
    #pragma unroll
                for (int k = 0; k < NSMAX; ++k)
    #pragma unroll
                    for (int c = 0; c < CNS; ++c) nsv[k][c] = nsp[static_cast<size_t>(c) * a.N + no[k]];
                __builtin_amdgcn_sched_barrier(0);
                {
                    T h[kQ];
    #pragma unroll
                    for (int i = 0; i < kQ; ++i) h[i] = ST::dec(rr[i], a.inv_scale);
                    reservoir_override(x, y, p, h);
                    s_rho[slot][s][me] = a.rho0[s] + sum19(h);
                    if (NC == 2 && js >= 0) {
                        s_j[js][s][0][tj] = first_moment<T, 0>(h);
                        s_j[js][s][1][tj] = first_moment<T, 1>(h);
                        s_j[js][s][2][tj] = first_moment<T, 2>(h);
                    }
    #pragma unroll
                    for (int i = 0; i < kQ; ++i) {
                        hz[i] = hs[i * NT_];
                        hs[i * NT_] = h[i];
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                issue(pn, qme, rr);
                __builtin_amdgcn_sched_barrier(0);
                if (ring) {
                    T hr[kQ];
    #pragma unroll
                    for (int i = 0; i < kQ; ++i) hr[i] = ST::dec(er[i], a.inv_scale);
                    reservoir_override(rx, ry, p, hr);
                    s_rho[slot][s][rme] = a.rho0[s] + sum19(hr);
                }
    #pragma unroll
                for (int k = 0; k < NSMAX; ++k)
    #pragma unroll
                    for (int c = 0; c < CNS; ++c) s_ns[slot][c][nl[k]] = nsv[k][c];
            };

            T hz[kQ];
            // prologue: plane zs-1 (densities only), plane zs (to hs)
            issue(wrapz(zs - 1), qme, rr);
            stage_pipe(wrapz(zs - 1), rslot(zs - 1), -1, zs, hz);
            stage_pipe(zs, rslot(zs), jslot(zs), wrapz(zs + 1), hz);
            for (int z = zs; z < ze; ++z) {
                // after the last plane the next loads repeat the one just staged (L2 hits)
                const int pn = z + 2 <= ze ? wrapz(z + 2) : wrapz(z + 1);
                stage_pipe(wrapz(z + 1), rslot(z + 1), jslot(z + 1), pn, hz);
                __syncthreads();
                collide(z, rslot(z - 1), rslot(z), rslot(z + 1), jslot(z), hz, false);
            }
        } else {
            // 16-bit storage: two roles, fixed per wave (NTC is a multiple of
            // 64, and the ring lanes are the first of each component).  Waves
            // holding ring lanes stage the ring densities as well and keep one
            // plane of own loads in flight; the others, free of the ring loads,
            // keep two (a wave has at most 63 memory operations outstanding,
            // and the 16-bit loads carry half the bytes each).  Both roles run
            // the same loop with one barrier per plane.  Wider formats keep one
            // role: there the deeper prefetch did not pay.
            constexpr bool kDeep = true;
            auto sweep = [&](auto ring_tag) {
                constexpr bool RING = decltype(ring_tag)::value;
                constexpr bool DEEP = kDeep && !RING;
                constexpr int AHEAD = DEEP ? 2 : 1;  // planes between issue and consumption
                E rA[kQ];
                E rB[DEEP ? kQ : 1];
                E er[RING ? kQ : 1];
                // Stage plane p, whose own loads are in rc: (ring loads and) n_s
                // are issued first; the own values give the density and first
                // moments and go to hs, whose previous content (the plane before)
                // moves to hz; then the own loads of plane pn are issued into rc,
                // and only after them the ring values are consumed, so a wait for
                // the ring does not wait for plane pn.
                auto stage_pipe = [&](int p, int slot, int js, int pn, T hz[kQ], E rc[kQ]) {
                    if constexpr (RING) issue(p, qr, er);
                    const float* nsp = ns + static_cast<size_t>(p) * plane;
                    float nsv[NSMAX][CNS];
    #pragma unroll
                    for (int k = 0; k < NSMAX; ++k)
    #pragma unroll
                        for (int c = 0; c < CNS; ++c) nsv[k][c] = nsp[static_cast<size_t>(c) * a.N + no[k]];
                    __builtin_amdgcn_sched_barrier(0);
                    {
                        T h[kQ];
    #pragma unroll
                        for (int i = 0; i < kQ; ++i) h[i] = ST::dec(rc[i], a.inv_scale);
                        reservoir_override(x, y, p, h);
                        s_rho[slot][s][me] = a.rho0[s] + sum19(h);
                        if (NC == 2 && js >= 0) {
                            s_j[js][s][0][tj] = first_moment<T, 0>(h);
                            s_j[js][s][1][tj] = first_moment<T, 1>(h);
                            s_j[js][s][2][tj] = first_moment<T, 2>(h);
                        }
    #pragma unroll
                        for (int i = 0; i < kQ; ++i) {
                            hz[i] = hs[i * NT_];
                            hs[i * NT_] = h[i];
                        }
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    issue(pn, qme, rc);
                    __builtin_amdgcn_sched_barrier(0);
                    if constexpr (RING) {
                        if (ring) {
                            T hr[kQ];
    #pragma unroll
                            for (int i = 0; i < kQ; ++i) hr[i] = ST::dec(er[i], a.inv_scale);
                            reservoir_override(rx, ry, p, hr);
                            s_rho[slot][s][rme] = a.rho0[s] + sum19(hr);
                        }
                    }
    #pragma unroll
                    for (int k = 0; k < NSMAX; ++k)
    #pragma unroll
                        for (int c = 0; c < CNS; ++c) s_ns[slot][c][nl[k]] = nsv[k][c];
                };
                // the plane whose loads a stage of plane p issues: p + AHEAD, or
                // after the last plane one already staged again (L2 hits)
                auto ahead = [&](int p) { return wrapz(p + AHEAD <= ze ? p + AHEAD : ze); };
                // register sets: planes zs-1, zs+1, ... in r_odd, planes zs, zs+2, ...
                // in r_even (one and the same set unless two planes are in flight)
                E (&r_odd)[kQ] = rA;
                E (&r_even)[kQ] = *reinterpret_cast<E(*)[kQ]>(DEEP ? static_cast<E*>(rB) : static_cast<E*>(rA));

                T hz[kQ];
                // prologue: planes zs-1 (densities only) and zs (to hs)
                issue(wrapz(zs - 1), qme, r_odd);
                if constexpr (DEEP) issue(zs, qme, r_even);
                stage_pipe(wrapz(zs - 1), rslot(zs - 1), -1, ahead(zs - 1), hz, r_odd);
                stage_pipe(zs, rslot(zs), jslot(zs), ahead(zs), hz, r_even);
                // unrolled by two so the register sets keep fixed names; every
                // wave, in either role, passes ze - zs barriers
                for (int z = zs; z < ze; z += 2) {
                    stage_pipe(wrapz(z + 1), rslot(z + 1), jslot(z + 1), ahead(z + 1), hz, r_odd);
                    __syncthreads();
                    collide(z, rslot(z - 1), rslot(z), rslot(z + 1), jslot(z), hz, false);
                    if (z + 1 >= ze) break;
                    stage_pipe(wrapz(z + 2), rslot(z + 2), jslot(z + 2), ahead(z + 2), hz, r_even);
                    __syncthreads();
                    collide(z + 1, rslot(z), rslot(z + 1), rslot(z + 2), jslot(z + 1), hz, false);
                }
            };
            const bool wave_ring = NC == 2 && __builtin_amdgcn_ballot_w64(ring) != 0;
            if (wave_ring) sweep(std::true_type{});
            else sweep(std::false_type{});
        }
    } else {
        T hA[kQ];
        T hB[kQ];

        // prologue: plane zs-1 (densities only), plane zs (kept in hA)
        stage_plane(wrapz(zs - 1), rslot(zs - 1), -1, hB);
        stage_plane(zs, rslot(zs), jslot(zs), hA);

        // sweep, two planes per iteration so the register sets alternate roles
        for (int z = zs; z < ze; z += 2) {
            stage_plane(wrapz(z + 1), rslot(z + 1), jslot(z + 1), hB);
            __syncthreads();
            collide(z, rslot(z - 1), rslot(z), rslot(z + 1), jslot(z), hA, true);
            if (z + 1 >= ze) break;
            stage_plane(wrapz(z + 2), rslot(z + 2), jslot(z + 2), hA);
            __syncthreads();
            collide(z + 1, rslot(z), rslot(z + 1), rslot(z + 2), jslot(z + 1), hB, true);
        }
    }
}

template <typename ST, int NC, int CNS, int TX, int TY, int FS, bool ONE>
__global__ __launch_bounds__(NC* TX* TY) void k_step(Args<typename ST::T> a,
                                                      const typename ST::E* __restrict__ A,
                                                      typename ST::E* __restrict__ B,
                                                      const float* __restrict__ ns)
{
    __shared__ TileShared<ST, NC, CNS, TX, TY> sh;
    // XCD-aware tile order: blocks are dispatched round-robin over 8 XCDs, so
    // give each XCD a contiguous run of tiles (neighbours share its L2).
    const int nb = gridDim.x;
    int L = blockIdx.x;
    if ((nb & 7) == 0) L = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
    step_tile<ST, NC, CNS, TX, TY, FS, ONE>(a, A, B, ns, L, a.t, sh);
}


// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// Batched step: the tiles of many domains in one launch.  The device table
// holds a header and one entry per domain (geometry, parameters, ping-pong
// buffers, steps to take in this tick, first tile index).  Blocks stride over
// the concatenated tile list, so the grid size does not depend on the mix and
// a captured graph of K launches (k = 0..K-1) stays valid when domains come
// and go: only the table changes.
template <typename T>
struct BatchEntry {
    Args<T> a;
    const void* buf[2];
    const float* ns;
    int parity;      // buffer holding the state at k = 0
    int steps;       // launches k < steps advance this domain
    int tile_begin;  // first tile of this domain in the concatenated list
    int ntiles;
};

struct BatchHeader {
    int ndom;
    int total_tiles;
    int pad[2];
};

constexpr size_t kBatchEntryOffset = 64;

template <typename ST, int NC, int CNS, int TX, int TY>
__global__ __launch_bounds__(NC* TX* TY) void k_step_batch(const char* __restrict__ table, int k)
{
    using T = typename ST::T;
    using E = typename ST::E;
    __shared__ TileShared<ST, NC, CNS, TX, TY> sh;
    const BatchHeader* hdr = reinterpret_cast<const BatchHeader*>(table);
    const BatchEntry<T>* ent = reinterpret_cast<const BatchEntry<T>*>(table + kBatchEntryOffset);
    const int total = hdr->total_tiles;
    const int nd = hdr->ndom;
    // XCD-aware order, as in k_step: blocks are dispatched round-robin over
    // the 8 XCDs, so give each XCD a contiguous run of every stride of tiles
    // (neighbouring tiles re-read each other's edge cells through its L2)
    const int nb = gridDim.x;
    const int b0 = (nb & 7) == 0 ? (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    for (int w = b0; w < total; w += nb) {
        int lo = 0, hi = nd - 1;  // last domain with tile_begin <= w
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (ent[mid].tile_begin <= w) lo = mid;
            else hi = mid - 1;
        }
        const BatchEntry<T>& e = ent[lo];
        if (k >= e.steps) continue;
        const int cur = (e.parity + k) & 1;
        __syncthreads();  // the previous tile's LDS is no longer read
        step_tile<ST, NC, CNS, TX, TY, kForcingShanChen>(e.a, static_cast<const E*>(e.buf[cur]), static_cast<E*>(const_cast<void*>(e.buf[1 - cur])),
                                       e.ns, w - e.tile_begin, e.a.t + static_cast<uint32_t>(k), sh);
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

// Electrolyte-filling diagnostics (Sec. 4) from the FP64 fields: per-block
// sums of p and cell counts over the inlet and outlet slabs (Eq. CapPressure),
// and of (1 - n_s) [rho_comp >= threshold] and (1 - n_s) over the pore slab
// (Eq. Saturation).
__global__ __launch_bounds__(kRedThreads) void k_fill(int nx, int ny, int nz, int N, FillQuery q, int ns_field,
                                                      const double* __restrict__ rho, const double* __restrict__ p,
                                                      const float* __restrict__ ns, double* __restrict__ partials)
{
    __shared__ double red[6][kRedThreads];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        const int x = n % nx, y = (n / nx) % ny, z = n / (nx * ny);
        const int c = q.axis == 0 ? x : (q.axis == 1 ? y : z);
        if (c >= q.inlet_lo && c < q.inlet_hi) {
            acc[0] += p[n];
            acc[1] += 1.0;
        }
        if (c >= q.outlet_lo && c < q.outlet_hi) {
            acc[2] += p[n];
            acc[3] += 1.0;
        }
        if (c >= q.pore_lo && c < q.pore_hi) {
            const double wfl = 1.0 - static_cast<double>(ns[static_cast<size_t>(ns_field) * N + n]);
            acc[4] += rho[static_cast<size_t>(q.comp) * N + n] >= q.threshold ? wfl : 0.0;
            acc[5] += wfl;
        }
    }
    for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 6) partials[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// Fixed-order sum of nblocks partials of K doubles each (one block): the
// result does not depend on timing.
template <int K>
__global__ __launch_bounds__(kRedThreads) void k_reduce(const double* __restrict__ partials, int nblocks,
                                                        double* __restrict__ out)
{
    __shared__ double red[K][kRedThreads];
    double acc[K];
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kRedThreads)
        for (int k = 0; k < K; ++k) acc[k] += partials[b * K + k];
    for (int k = 0; k < K; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < K; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < K) out[threadIdx.x] = red[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// Launchers.

bool tile_supported(int tx, int ty)
{
    return (tx == 128 && ty == 4) || (tx == 64 && (ty == 4 || ty == 8)) || (tx == 32 && (ty == 4 || ty == 8 || ty == 16));
}

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

template <typename ST, int NC, int CNS, int TX, int TY, int FS, bool ONE>
static hipError_t step_t(const Problem& p, const Launch& l, int64_t t, const void* A, void* B, const float* ns,
                         hipStream_t st)
{
    using T = typename ST::T;
    using E = typename ST::E;
    Args<T> a = make_args<T>(p);
    a.zchunk = l.zchunk;
    a.ntx = (p.nx + TX - 1) / TX;
    a.nty = (p.ny + TY - 1) / TY;
    a.nzc = (p.nz + l.zchunk - 1) / l.zchunk;
    a.t = static_cast<uint32_t>(t);
    const int nblocks = a.ntx * a.nty * a.nzc;
    hipLaunchKernelGGL((k_step<ST, NC, CNS, TX, TY, FS, ONE>), dim3(nblocks), dim3(NC * TX * TY), 0, st, a,
                       static_cast<const E*>(A), static_cast<E*>(B), ns);
    return hipGetLastError();
}

// Tile shapes (TX x TY cells per block) compiled in.
template <typename ST, int NC, int CNS>
static hipError_t step_ty(const Problem& p, const Launch& l, int64_t t, const void* A, void* B, const float* ns,
                          hipStream_t st)
{
    constexpr int SC = kForcingShanChen, GUO = kForcingGuo;
    // one-cell-deep domains on the default tiles: the one-plane instances
    const bool one = p.nz == 1;
    if (p.forcing == kForcingGuo) {  // the GS-WBS: the default tiles only
        if (l.tile_x == 64 && l.tile_y == 8)
            return one ? step_t<ST, NC, CNS, 64, 8, GUO, true>(p, l, t, A, B, ns, st)
                       : step_t<ST, NC, CNS, 64, 8, GUO, false>(p, l, t, A, B, ns, st);
        if (l.tile_x == 64 && l.tile_y == 4)
            return one ? step_t<ST, NC, CNS, 64, 4, GUO, true>(p, l, t, A, B, ns, st)
                       : step_t<ST, NC, CNS, 64, 4, GUO, false>(p, l, t, A, B, ns, st);
        return hipErrorInvalidValue;
    }
    if (l.tile_x == 64 && l.tile_y == 8)
        return one ? step_t<ST, NC, CNS, 64, 8, SC, true>(p, l, t, A, B, ns, st)
                   : step_t<ST, NC, CNS, 64, 8, SC, false>(p, l, t, A, B, ns, st);
    if (l.tile_x == 64 && l.tile_y == 4)
        return one ? step_t<ST, NC, CNS, 64, 4, SC, true>(p, l, t, A, B, ns, st)
                   : step_t<ST, NC, CNS, 64, 4, SC, false>(p, l, t, A, B, ns, st);
    if (l.tile_x == 128 && l.tile_y == 4) return step_t<ST, NC, CNS, 128, 4, SC, false>(p, l, t, A, B, ns, st);
    if (l.tile_x == 32 && l.tile_y == 4) return step_t<ST, NC, CNS, 32, 4, SC, false>(p, l, t, A, B, ns, st);
    if (l.tile_x == 32 && l.tile_y == 8) return step_t<ST, NC, CNS, 32, 8, SC, false>(p, l, t, A, B, ns, st);
    if (l.tile_x == 32 && l.tile_y == 16) return step_t<ST, NC, CNS, 32, 16, SC, false>(p, l, t, A, B, ns, st);
    return hipErrorInvalidValue;
}

template <typename ST>
static hipError_t step_st(const Problem& p, const Launch& l, int64_t t, const void* A, void* B, const float* ns,
                          hipStream_t st)
{
    if (p.ncomp == 1) return step_ty<ST, 1, 1>(p, l, t, A, B, ns, st);
    if (p.c_ns == 1) return step_ty<ST, 2, 1>(p, l, t, A, B, ns, st);
    return step_ty<ST, 2, 2>(p, l, t, A, B, ns, st);
}

hipError_t launch_step(const Problem& p, const Launch& l, int64_t t, const void* A, void* B, const float* ns,
                       hipStream_t st)
{
    switch (p.storage) {
    case kF64: return step_st<F64>(p, l, t, A, B, ns, st);
    case kF32: return step_st<F32>(p, l, t, A, B, ns, st);
    case kF16: return step_st<F16>(p, l, t, A, B, ns, st);
    case kBF16: return step_st<BF16>(p, l, t, A, B, ns, st);
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
    hipLaunchKernelGGL(k_reduce<5>, dim3(1), dim3(kRedThreads), 0, st, partials, nblocks, out);
    return hipGetLastError();
}

hipError_t launch_fill(const Problem& p, const FillQuery& q, const double* rho, const double* pr, const float* ns,
                       double* partials, double* out, hipStream_t st)
{
    const int nb = static_cast<int>(std::min<int64_t>(moments_max_blocks(), (p.N + kRedThreads - 1) / kRedThreads));
    const int ns_field = p.c_ns == 2 ? q.comp : 0;
    hipLaunchKernelGGL(k_fill, dim3(nb), dim3(kRedThreads), 0, st, p.nx, p.ny, p.nz, static_cast<int>(p.N), q,
                       ns_field, rho, pr, ns, partials);
    hipLaunchKernelGGL(k_reduce<6>, dim3(1), dim3(kRedThreads), 0, st, partials, nb, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched launches.

template <typename T>
static size_t batch_bytes_t(int max_domains)
{
    return kBatchEntryOffset + sizeof(BatchEntry<T>) * static_cast<size_t>(max_domains > 0 ? max_domains : 1);
}

size_t batch_table_bytes(int storage, int max_domains)
{
    return storage == kF64 ? batch_bytes_t<double>(max_domains) : batch_bytes_t<float>(max_domains);
}

template <typename T>
static int batch_encode_t(const BatchDomain* d, int n, int tile_x, int tile_y, void* host)
{
    BatchHeader* h = static_cast<BatchHeader*>(host);
    BatchEntry<T>* e = reinterpret_cast<BatchEntry<T>*>(static_cast<char*>(host) + kBatchEntryOffset);
    int tiles = 0;
    for (int i = 0; i < n; ++i) {
        Args<T> a = make_args<T>(d[i].prob);
        a.zchunk = d[i].zchunk;
        a.ntx = (d[i].prob.nx + tile_x - 1) / tile_x;
        a.nty = (d[i].prob.ny + tile_y - 1) / tile_y;
        a.nzc = (d[i].prob.nz + a.zchunk - 1) / a.zchunk;
        a.t = static_cast<uint32_t>(d[i].t);
        e[i].a = a;
        e[i].buf[0] = d[i].buf[0];
        e[i].buf[1] = d[i].buf[1];
        e[i].ns = d[i].ns;
        e[i].parity = d[i].parity;
        e[i].steps = d[i].steps;
        e[i].tile_begin = tiles;
        e[i].ntiles = a.ntx * a.nty * a.nzc;
        tiles += e[i].ntiles;
    }
    h->ndom = n;
    h->total_tiles = tiles;
    h->pad[0] = h->pad[1] = 0;
    return tiles;
}

int batch_encode(int storage, const BatchDomain* d, int n, int tile_x, int tile_y, void* host)
{
    return storage == kF64 ? batch_encode_t<double>(d, n, tile_x, tile_y, host)
                           : batch_encode_t<float>(d, n, tile_x, tile_y, host);
}

template <typename ST, int NC, int CNS, int TX, int TY>
static hipError_t batch_t(const void* table, int k, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_step_batch<ST, NC, CNS, TX, TY>), dim3(grid), dim3(NC * TX * TY), 0, st,
                       static_cast<const char*>(table), k);
    return hipGetLastError();
}

template <typename ST, int NC, int CNS>
static hipError_t batch_tile(int tx, int ty, const void* table, int k, int grid, hipStream_t st)
{
    if (tx == 64 && ty == 8) return batch_t<ST, NC, CNS, 64, 8>(table, k, grid, st);
    if (tx == 32 && ty == 8) return batch_t<ST, NC, CNS, 32, 8>(table, k, grid, st);
    return hipErrorInvalidValue;
}

template <typename ST>
static hipError_t batch_st(int ncomp, int c_ns, int tx, int ty, const void* table, int k, int grid, hipStream_t st)
{
    if (ncomp == 1) return batch_tile<ST, 1, 1>(tx, ty, table, k, grid, st);
    if (c_ns == 1) return batch_tile<ST, 2, 1>(tx, ty, table, k, grid, st);
    return batch_tile<ST, 2, 2>(tx, ty, table, k, grid, st);
}

bool batch_tile_supported(int tx, int ty) { return (tx == 64 && ty == 8) || (tx == 32 && ty == 8); }

template <typename ST, int NC, int CNS, int TX, int TY>
static int batch_occ_t()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_batch<ST, NC, CNS, TX, TY>, NC * TX * TY, 0) !=
        hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

template <typename ST, int NC, int CNS>
static int batch_occ_tile(int tx, int ty)
{
    if (tx == 64 && ty == 8) return batch_occ_t<ST, NC, CNS, 64, 8>();
    if (tx == 32 && ty == 8) return batch_occ_t<ST, NC, CNS, 32, 8>();
    return 1;
}

template <typename ST>
static int batch_occ_st(int ncomp, int c_ns, int tx, int ty)
{
    if (ncomp == 1) return batch_occ_tile<ST, 1, 1>(tx, ty);
    if (c_ns == 1) return batch_occ_tile<ST, 2, 1>(tx, ty);
    return batch_occ_tile<ST, 2, 2>(tx, ty);
}

int batch_blocks_per_cu(int storage, int ncomp, int c_ns, int tile_x, int tile_y)
{
    switch (storage) {
    case kF64: return batch_occ_st<F64>(ncomp, c_ns, tile_x, tile_y);
    case kF32: return batch_occ_st<F32>(ncomp, c_ns, tile_x, tile_y);
    case kF16: return batch_occ_st<F16>(ncomp, c_ns, tile_x, tile_y);
    case kBF16: return batch_occ_st<BF16>(ncomp, c_ns, tile_x, tile_y);
    default: return 1;
    }
}

hipError_t launch_step_batch(int storage, int ncomp, int c_ns, int tile_x, int tile_y, const void* table, int k,
                             int grid, hipStream_t st)
{
    switch (storage) {
    case kF64: return batch_st<F64>(ncomp, c_ns, tile_x, tile_y, table, k, grid, st);
    case kF32: return batch_st<F32>(ncomp, c_ns, tile_x, tile_y, table, k, grid, st);
    case kF16: return batch_st<F16>(ncomp, c_ns, tile_x, tile_y, table, k, grid, st);
    case kBF16: return batch_st<BF16>(ncomp, c_ns, tile_x, tile_y, table, k, grid, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hm
