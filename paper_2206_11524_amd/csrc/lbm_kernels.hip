// HIP kernels (gfx950) of the HMCSC lattice Boltzmann update.
//
// Layout in HBM: populations are grouped by plane.  For one component the 19
// direction arrays of plane z lie next to each other, P[((s*nz + z)*19 + i)*
// plane + n], n = y*nx + x the in-plane index ("split" layout, FP64 and
// single-component runs).  Two-component runs in FP32 and the 16-bit formats
// keep the two components of one (cell, direction) in one word (64 or 32
// bits), P[(((z*19 + i)*plane + n) << 1) + s] ("pair" layout), so one load
// brings both.
// Streaming is "pull": a buffer holds the populations that left each cell at
// the previous step, so the pre-collision state of Eq. (LGS) at cell x is
// f_i(x) = P_i(x - c_i) (periodic).  Every stored value is shifted,
// h = f - w_i*rho0_s (scaled by 2^k for the 16-bit formats); the whole
// collision is written in the shifted variables (the shift cancels in the
// partial bounce-back blend because w_ibar = w_i), which keeps small deviations
// representable in reduced precision.
//
// The step kernels are fused 2.5-D sweeps: a block owns a TX x TY column of
// cells and marches along z.  For every plane it pulls the populations of its
// cells once (kept for the collision of a later iteration), forms the
// densities, and stages them in LDS together with a one-cell ring of densities
// recomputed from the ring cells' populations, plus the n_s field.  The
// cohesion force (Eq. SC_F_inter) and adhesion force (Eq. SC_F_ads) then read
// their 18 neighbours from LDS, so HBM sees each population read once and
// written once per step (ring and z-halo re-reads hit L2/MALL).  Every plane
// is addressed through its own buffer descriptor (base = start of the plane
// block, 64-bit, built on the scalar unit), so no 32-bit offset spans more
// than one plane and domains of any size that fits the device are addressed.
#include "lbm_kernels.h"

#include <stdint.h>

#include <algorithm>
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
    // Stochastic rounding with the random word r (v_cvt_sr_f16_f32): the
    // instruction reads its random operand as a binary fraction from the top
    // bit down and rounds the magnitude up with probability equal to the
    // value's fraction of the binary16 spacing, subnormals included (checked
    // on the device: up only for bit 31 at half a spacing, frequencies equal
    // to the fraction, exact values unchanged, inf and NaN kept).  The top 16
    // bits of r are random (see lcg24), so the probability is resolved to
    // 2^-16.
    static __device__ __forceinline__ E enc_sr(T v, T scale, uint32_t r)
    {
        half2_t h = {0, 0};
        h = __builtin_amdgcn_cvt_sr_f16_f32(h, v * scale, r, false);
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
    // round to nearest, ties to even (gfx950's v_cvt_pk_bf16_f32)
    static __device__ __forceinline__ E enc(T v, T scale)
    {
        return __builtin_bit_cast(uint16_t, static_cast<__bf16>(v * scale));
    }
    // Stochastic rounding with the random word r (v_cvt_sr_bf16_f32, the same
    // convention as the binary16 instruction).
    static __device__ __forceinline__ E enc_sr(T v, T scale, uint32_t r)
    {
        bf162_t h = {0, 0};
        h = __builtin_amdgcn_cvt_sr_bf16_f32(h, v * scale, r, false);
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

// The following random words of one (cell, component), after fmix32 has
// seeded them: a linear congruential step modulo 2^24 (multiplier = 1 mod 4,
// odd increment: full period by Hull and Dobell's conditions) on the low 24
// bits of the previous word, kept as the 32-bit value a*x + c, whose top 16
// bits the rounding reads.  One 24-bit multiply-add (v_mad_u32_u24) per
// stored value.
constexpr uint32_t kLcgA = 0x6d2b79u, kLcgC = 0x2b5a3fu;
static_assert(kLcgA % 4 == 1 && kLcgC % 2 == 1 && kLcgA < (1u << 24), "full-period LCG modulo 2^24");
__device__ __forceinline__ uint32_t lcg24(uint32_t x) { return (x & 0xffffffu) * kLcgA + kLcgC; }

// Two 16-bit values of one (cell, direction) in one 32-bit word of the pair
// layout: component 0 in the low half, component 1 in the high half.  The
// pair kernel works on the stored scale (h * 2^k): the power-of-two factor
// is folded into the few per-cell coefficients instead of every value, which
// changes no bit (scaling by 2^k commutes with rounding).
template <typename ST>
struct PairCodec {
    static __device__ __forceinline__ float lo(uint32_t v) { return ST::dec(static_cast<uint16_t>(v & 0xffffu), 1.0f); }
    static __device__ __forceinline__ float hi(uint32_t v) { return ST::dec(static_cast<uint16_t>(v >> 16), 1.0f); }
    // x_H + y_H and x_H - y_H for the halves H (0 low, 1 high) of two words,
    // each rounded once to FP32.  Binary16: one v_fma_mix_f32 (x * 1 + y with
    // both sources converted from binary16 inside the instruction) instead of
    // two conversions and an add; the result is the same, as the conversions
    // are exact.  bfloat16 decodes with one shift or mask per value anyway.
    template <int H>
    static __device__ __forceinline__ float sum(uint32_t x, uint32_t y)
    {
        if constexpr (std::is_same_v<ST, F16>) {
            float r;
            if constexpr (H == 0)
                asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(x), "v"(y));
            else
                asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(x), "v"(y));
            return r;
        } else {
            return H == 0 ? lo(x) + lo(y) : hi(x) + hi(y);
        }
    }
    template <int H>
    static __device__ __forceinline__ float diff(uint32_t x, uint32_t y)
    {
        if constexpr (std::is_same_v<ST, F16>) {
            float r;
            if constexpr (H == 0)
                asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel_hi:[1,0,1]" : "=v"(r) : "v"(x), "v"(y));
            else
                asm("v_fma_mix_f32 %0, %1, 1.0, -%2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(x), "v"(y));
            return r;
        } else {
            return H == 0 ? lo(x) - lo(y) : hi(x) - hi(y);
        }
    }
    static __device__ __forceinline__ uint32_t enc(float a, float b)
    {
        if constexpr (std::is_same_v<ST, BF16>) {
            const bf162_t h = {static_cast<__bf16>(a), static_cast<__bf16>(b)};
            return __builtin_bit_cast(uint32_t, h);
        } else {
            const half2_t h = {static_cast<_Float16>(a), static_cast<_Float16>(b)};
            return __builtin_bit_cast(uint32_t, h);
        }
    }
    // stochastic rounding (see F16::enc_sr) of a into the low and b into the
    // high half of one word, with the random words ra and rb
    static __device__ __forceinline__ uint32_t enc_sr(float a, float b, uint32_t ra, uint32_t rb)
    {
        if constexpr (std::is_same_v<ST, BF16>) {
            bf162_t h = {0, 0};
            h = __builtin_amdgcn_cvt_sr_bf16_f32(h, a, ra, false);
            h = __builtin_amdgcn_cvt_sr_bf16_f32(h, b, rb, true);
            return __builtin_bit_cast(uint32_t, h);
        } else {
            half2_t h = {0, 0};
            h = __builtin_amdgcn_cvt_sr_f16_f32(h, a, ra, false);
            h = __builtin_amdgcn_cvt_sr_f16_f32(h, b, rb, true);
            return __builtin_bit_cast(uint32_t, h);
        }
    }
};

// FP32 pair words: component 0 in the low, component 1 in the high 32 bits
// (stored as they are, rounded to nearest by the collision's arithmetic).
template <>
struct PairCodec<F32> {
    static __device__ __forceinline__ float lo(u32x2 v) { return __uint_as_float(v.x); }
    static __device__ __forceinline__ float hi(u32x2 v) { return __uint_as_float(v.y); }
    template <int H>
    static __device__ __forceinline__ float sum(u32x2 x, u32x2 y)
    {
        return H == 0 ? lo(x) + lo(y) : hi(x) + hi(y);
    }
    template <int H>
    static __device__ __forceinline__ float diff(u32x2 x, u32x2 y)
    {
        return H == 0 ? lo(x) - lo(y) : hi(x) - hi(y);
    }
    static __device__ __forceinline__ u32x2 enc(float a, float b)
    {
        u32x2 w;
        w.x = __float_as_uint(a);
        w.y = __float_as_uint(b);
        return w;
    }
};

// Word of the pair layout: both components of one (cell, direction), 32 bits
// for the 16-bit formats, 64 bits for FP32.
template <typename ST>
struct PairWordOf {
    using W = uint32_t;
};
template <>
struct PairWordOf<F32> {
    using W = u32x2;
};

template <typename W>
__device__ __forceinline__ W word_load(rsrc_t r, uint32_t vo, uint32_t so)
{
    if constexpr (sizeof(W) == 8) return __builtin_bit_cast(W, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
    else return __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0);
}

template <typename W>
__device__ __forceinline__ void word_store(W v, rsrc_t r, uint32_t vo, uint32_t so)
{
    if constexpr (sizeof(W) == 8) __builtin_amdgcn_raw_buffer_store_b64(v, r, vo, so, kNT);
    else __builtin_amdgcn_raw_buffer_store_b32(v, r, vo, so, kNT);
}

// Kernel parameters in the arithmetic type.
template <typename T>
struct Args {
    int nx, ny, nz;
    int plane;   // nx * ny
    int64_t N;   // cells
    int pair;    // populations in the pair layout
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
    a.plane = p.nx * p.ny;
    a.N = p.N;
    a.pair = pair_layout(p.storage, p.ncomp, p.forcing) ? 1 : 0;
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

// Element index of population (component s, direction i) of in-plane cell n of
// plane z, in either layout (auxiliary kernels; the step kernels address whole
// plane blocks through buffer descriptors).
template <typename T>
__device__ __forceinline__ size_t pidx(const Args<T>& a, int s, int i, int z, int64_t n)
{
    if (a.pair) return (((static_cast<size_t>(z) * kQ + i) * static_cast<size_t>(a.plane) + n) << 1) + s;
    return ((static_cast<size_t>(s) * a.nz + z) * kQ + i) * static_cast<size_t>(a.plane) + n;
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

// Both components at once (pair kernel).
template <typename T>
__device__ __forceinline__ bool reservoir_dr2(const Args<T>& a, int x, int y, int z, T& dr0, T& dr1)
{
    bool in = false;
    dr0 = T(0);
    dr1 = T(0);
#pragma unroll
    for (int r = 0; r < kMaxRes; ++r) {
        if (r < a.n_res) {
            const int c = a.res_axis[r] == 0 ? x : (a.res_axis[r] == 1 ? y : z);
            const bool hit = !in && c >= a.res_lo[r] && c < a.res_hi[r];
            dr0 = hit ? a.res_dr[r][0] : dr0;
            dr1 = hit ? a.res_dr[r][1] : dr1;
            in = in || hit;
        }
    }
    return in;
}

// Reservoir membership as bit masks (pair kernel): bit r is set when the cell
// lies in slot r.  Slots along x or y depend on the cell's column only, so a
// thread computes their bits once; slots along z depend on the plane only, the
// same for the whole block.  The lowest set bit is the slot that applies
// (slots are searched in order, as in reservoir_dr).
template <typename T>
__device__ __forceinline__ uint32_t reservoir_xy_bits(const Args<T>& a, int x, int y)
{
    uint32_t m = 0;
#pragma unroll
    for (int r = 0; r < kMaxRes; ++r) {
        const int c = a.res_axis[r] == 0 ? x : y;
        if (r < a.n_res && a.res_axis[r] != 2 && c >= a.res_lo[r] && c < a.res_hi[r]) m |= 1u << r;
    }
    return m;
}

template <typename T>
__device__ __forceinline__ uint32_t reservoir_z_bits(const Args<T>& a, int z)
{
    uint32_t m = 0;
#pragma unroll
    for (int r = 0; r < kMaxRes; ++r)
        if (r < a.n_res && a.res_axis[r] == 2 && z >= a.res_lo[r] && z < a.res_hi[r]) m |= 1u << r;
    return m;
}

// shifted densities of the slot of the lowest bit of m (m != 0)
template <typename T>
__device__ __forceinline__ void reservoir_pick(const Args<T>& a, uint32_t m, T& dr0, T& dr1)
{
    dr0 = a.res_dr[kMaxRes - 1][0];
    dr1 = a.res_dr[kMaxRes - 1][1];
#pragma unroll
    for (int r = kMaxRes - 2; r >= 0; --r) {
        const bool hit = (m >> r) & 1u;
        dr0 = hit ? a.res_dr[r][0] : dr0;
        dr1 = hit ? a.res_dr[r][1] : dr1;
    }
}

__device__ __forceinline__ int wrap_dec(int v, int n) { return v == 0 ? n - 1 : v - 1; }
__device__ __forceinline__ int wrap_inc(int v, int n) { return v == n - 1 ? 0 : v + 1; }

// In-plane byte offsets of the nine (x - cx, y - cy) sources of a cell, for
// elements of EB bytes.
struct PlaneOffs {
    uint32_t o[3][3];  // [cy + 1][cx + 1]
};

template <int EB>
__device__ __forceinline__ PlaneOffs plane_offs(int x, int y, int nx, int ny)
{
    const int xs[3] = {x == nx - 1 ? 0 : x + 1, x, x == 0 ? nx - 1 : x - 1};  // x - c, c = -1, 0, 1
    const int ys[3] = {y == ny - 1 ? 0 : y + 1, y, y == 0 ? ny - 1 : y - 1};
    PlaneOffs q;
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) q.o[b][a] = static_cast<uint32_t>(ys[b] * nx + xs[a]) * static_cast<uint32_t>(EB);
    return q;
}

// Pull loads of one cell (raw stored values): direction i comes from the
// source plane z - c_iz, whose block descriptor is r3[c_iz + 1], at the
// in-plane offset of (x - c_ix, y - c_iy) plus i direction strides.
template <typename ST>
__device__ __forceinline__ void pull_raw(const rsrc_t r3[3], uint32_t dir_bytes, const PlaneOffs& q,
                                         typename ST::E e[kQ])
{
#pragma unroll
    for (int i = 0; i < kQ; ++i)
        e[i] = ST::bld(r3[CZ[i] + 1], q.o[CY[i] + 1][CX[i] + 1], static_cast<uint32_t>(i) * dir_bytes);
}

template <typename ST, typename T>
__device__ __forceinline__ void pull(const rsrc_t r3[3], uint32_t dir_bytes, const PlaneOffs& q, T inv_scale,
                                     T h[kQ])
{
#pragma unroll
    for (int i = 0; i < kQ; ++i)
        h[i] = ST::dec(ST::bld(r3[CZ[i] + 1], q.o[CY[i] + 1][CX[i] + 1], static_cast<uint32_t>(i) * dir_bytes),
                       inv_scale);
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

// Both components of one cell (pair kernel): the equilibrium velocities of
// Eq. (SC_u_eq) for s = 0 and 1, with the same expressions, in the same order,
// as cell_velocity evaluates for each component, so a cell's result does not
// depend on which kernel updated it.  The adhesion stencil of a single n_s
// field is shared by the two components.
template <int CNS, int LW, int LP>
__device__ __forceinline__ void cell_velocity_pair(const Args<float>& a, int me, const float* rho_m,
                                                   const float* rho_0, const float* rho_p, const float* ns_m,
                                                   const float* ns_0, const float* ns_p, const float (&jc)[2][3],
                                                   float ueq[2][3], float rho_own[2], float n[2])
{
    using T = float;
    T rho = 0, den = 0, num[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const T rc = rho_0[c * LP + me];
        rho_own[c] = rc;
        rho += rc;
        den += rc * a.inv_tau[c];
#pragma unroll
        for (int d = 0; d < 3; ++d) num[d] += jc[c][d] * a.inv_tau[c];
    }
    const T inv_den = den > T(0) ? recip(den) : T(0);
    const T inv_rho = rho > T(0) ? recip(rho) : T(0);
    // one stencil at a time (a scheduling fence after each): all 54 or 72
    // neighbour reads in flight at once would need as many registers
    T ga[CNS][3];
#pragma unroll
    for (int cn = 0; cn < CNS; ++cn) {
        stencil<T, float, LW>(ns_m + cn * LP, ns_0 + cn * LP, ns_p + cn * LP, me, ga[cn]);
        __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int cn = CNS == 2 ? s : 0;
        T gi[3];
        stencil<T, T, LW>(rho_m + (1 - s) * LP, rho_0 + (1 - s) * LP, rho_p + (1 - s) * LP, me, gi);
        __builtin_amdgcn_sched_barrier(0);
        const bool present = rho_own[s] > T(0);
        const T tau_s = a.tau[s], Gads = a.Gads_s[s];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const T acc = -a.G_s * gi[d] - Gads * ga[cn][d] + a.F[d] * inv_rho;
            ueq[s][d] = num[d] * inv_den + (present ? tau_s * acc : T(0));
        }
        n[s] = static_cast<T>(ns_0[cn * LP + me]);
    }
}

// The GS-WBS for both components of one cell: u_macro of Eq. (HMCSC_u_macro)
// and each component's total force, as cell_velocity_guo computes them.
template <int CNS, int LW, int LP>
__device__ __forceinline__ void cell_velocity_guo_pair(const Args<float>& a, int me, const float* rho_m,
                                                       const float* rho_0, const float* rho_p, const float* ns_m,
                                                       const float* ns_0, const float* ns_p,
                                                       const float (&jc)[2][3], float um[3], float fo[2][3],
                                                       float rho_own[2], float n_own[2])
{
    using T = float;
    T rc[2], rho = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        rc[c] = rho_0[c * LP + me];
        rho += rc[c];
    }
    const T inv_rho = rho > T(0) ? recip(rho) : T(0);
    T m[3] = {0, 0, 0};
    T ga[3];
    if constexpr (CNS == 1) stencil<T, float, LW>(ns_m, ns_0, ns_p, me, ga);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int cn = CNS == 2 ? c : 0;
        if constexpr (CNS == 2) stencil<T, float, LW>(ns_m + cn * LP, ns_0 + cn * LP, ns_p + cn * LP, me, ga);
        T gi[3];
        stencil<T, T, LW>(rho_m + (1 - c) * LP, rho_0 + (1 - c) * LP, rho_p + (1 - c) * LP, me, gi);
        const T nc = static_cast<T>(ns_0[cn * LP + me]);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            fo[c][d] = rc[c] * (-a.G_s * gi[d] - a.Gads_s[c] * ga[d] + a.F[d] * inv_rho);
            m[d] += (T(1) - nc) * (jc[c][d] + T(0.5) * fo[c][d]);
        }
        rho_own[c] = rc[c];
        n_own[c] = nc;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) um[d] = m[d] * inv_rho;
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
    const PlaneOffs qme = plane_offs<sizeof(E)>(x, y, a.nx, a.ny);
    const uint32_t own = static_cast<uint32_t>(y * a.nx + x) * static_cast<uint32_t>(sizeof(E));

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
    const PlaneOffs qring = plane_offs<sizeof(E)>(rx, ry, a.nx, a.ny);

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

    // The 19 direction arrays of one plane of this component form a block;
    // each plane block is addressed through its own buffer descriptor (64-bit
    // base on the scalar unit, 32-bit offsets within the block).
    const size_t cstride = static_cast<size_t>(a.nz) * kQ * static_cast<size_t>(plane);
    const E* Ac = A + static_cast<size_t>(s) * cstride;
    E* Bc = B + static_cast<size_t>(s) * cstride;
    const uint32_t dir_bytes = static_cast<uint32_t>(plane) * static_cast<uint32_t>(sizeof(E));
    const uint32_t blk_bytes = static_cast<uint32_t>(kQ) * dir_bytes;
    auto blk = [&](const E* base, int p) {
        return make_rsrc(base + static_cast<size_t>(p) * kQ * static_cast<size_t>(plane), blk_bytes);
    };

    auto pull_plane = [&](int p, const PlaneOffs& q, T h[kQ]) {
        const rsrc_t r3[3] = {blk(Ac, wrapz(p + 1)), blk(Ac, p), blk(Ac, wrapz(p - 1))};  // c_z = -1, 0, +1
        pull<ST, T>(r3, dir_bytes, q, a.inv_scale, h);
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
        const rsrc_t rz = blk(Bc, z);
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
            // one random word per stored value: fmix32 of (cell, component,
            // time step) for the rest population, then lcg24 steps in the
            // order of the stores
            const uint32_t cell = static_cast<uint32_t>(z) * static_cast<uint32_t>(plane) + static_cast<uint32_t>(y * a.nx + x);
            uint32_t r = fmix32(t_key ^ (2u * cell + static_cast<uint32_t>(s)));
            ST::bst(ST::enc_sr(rest(), a.scale, r), rz, own, 0u);
#pragma unroll
            for (int i = 1; i <= 9; ++i) {
                T pi, po;
                pair(i, pi, po);
                r = lcg24(r);
                ST::bst(ST::enc_sr(pi, a.scale, r), rz, own, static_cast<uint32_t>(i) * dir_bytes);
                r = lcg24(r);
                ST::bst(ST::enc_sr(po, a.scale, r), rz, own, static_cast<uint32_t>(i + 9) * dir_bytes);
            }
        } else {
            ST::bst(ST::enc(rest(), a.scale), rz, own, 0u);
#pragma unroll
            for (int i = 1; i <= 9; ++i) {
                T pi, po;
                pair(i, pi, po);
                ST::bst(ST::enc(pi, a.scale), rz, own, static_cast<uint32_t>(i) * dir_bytes);
                ST::bst(ST::enc(po, a.scale), rz, own, static_cast<uint32_t>(i + 9) * dir_bytes);
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
        // without a ring cell load the tile's last ring cell (a cell of the
        // domain; the values are not used), and lanes without an n_s cell
        // duplicate cell 0 of the staging list.
        constexpr int NT_ = TileShared<ST, NC, CNS, TX, TY>::NT;
        T* hs = &sh.hs[0][0] + threadIdx.x;
        const PlaneOffs& qr = qring;
        // list cell 0 is the corner (x0 - 1, y0 - 1), LDS index 0
        const int ns_off0 = (((y0 - 1) % a.ny + a.ny) % a.ny) * a.nx + ((x0 - 1) % a.nx + a.nx) % a.nx;
        int nl[NSMAX], no[NSMAX];
#pragma unroll
        for (int k = 0; k < NSMAX; ++k) {
            nl[k] = ns_lds[k] >= 0 ? ns_lds[k] : 0;
            no[k] = ns_lds[k] >= 0 ? ns_off[k] : ns_off0;
        }
        auto issue = [&](int p, const PlaneOffs& q, E e[kQ]) {
            const rsrc_t r3[3] = {blk(Ac, wrapz(p + 1)), blk(Ac, p), blk(Ac, wrapz(p - 1))};
            pull_raw<ST>(r3, dir_bytes, q, e);
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
        if constexpr (sizeof(E) == 8 || (sizeof(E) == 4 && FS == kForcingGuo)) {
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
            // One component in FP32 or a 16-bit format (two components run
            // the pair kernel): no ring, and in 16-bit two planes of own loads
            // in flight (a wave has at most 63 memory operations outstanding,
            // and the 16-bit loads carry half the bytes each; for FP32 the
            // deeper prefetch did not pay).
            static_assert(NC == 1, "two components in FP32 or 16-bit run the pair kernel");
            constexpr bool DEEP = sizeof(E) == 2;
            constexpr int AHEAD = DEEP ? 2 : 1;  // planes between issue and consumption
            E rA[kQ];
            E rB[DEEP ? kQ : 1];
            // Stage plane p, whose own loads are in rc: the n_s loads are
            // issued first; the own values give the density and go to hs,
            // whose previous content (the plane before) moves to hz; then the
            // own loads of plane pn are issued into rc.
            auto stage_pipe = [&](int p, int slot, int pn, T hz[kQ], E rc[kQ]) {
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
#pragma unroll
                    for (int i = 0; i < kQ; ++i) {
                        hz[i] = hs[i * NT_];
                        hs[i * NT_] = h[i];
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
                issue(pn, qme, rc);
                __builtin_amdgcn_sched_barrier(0);
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
            stage_pipe(wrapz(zs - 1), rslot(zs - 1), ahead(zs - 1), hz, r_odd);
            stage_pipe(zs, rslot(zs), ahead(zs), hz, r_even);
            // unrolled by two so the register sets keep fixed names
            for (int z = zs; z < ze; z += 2) {
                stage_pipe(wrapz(z + 1), rslot(z + 1), ahead(z + 1), hz, r_odd);
                __syncthreads();
                collide(z, rslot(z - 1), rslot(z), rslot(z + 1), jslot(z), hz, false);
                if (z + 1 >= ze) break;
                stage_pipe(wrapz(z + 2), rslot(z + 2), ahead(z + 2), hz, r_even);
                __syncthreads();
                collide(z + 1, rslot(z), rslot(z + 1), rslot(z + 2), jslot(z + 1), hz, false);
            }
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

// ---------------------------------------------------------------------------
// Pair kernel: two components in FP32 or a 16-bit format, one thread per cell.
//
// In the pair layout one word (32 bits for the 16-bit formats, 64 for FP32)
// holds both components' value of one (cell, direction), so a thread pulls
// its cell's 38 populations with 19 loads and stores them with 19 stores.
// Per memory operation that moves twice the bytes of a lone value, which
// doubles the bytes a wave keeps in flight under the same limit on
// outstanding operations and halves the memory instructions per cell.  The two
// components of a cell meet in registers, so the first moments need no LDS
// exchange; the densities still go to LDS for the force stencils.
//
// The waves of a block have fixed roles.  The first TX*TY threads own one
// cell each: they pull, collide and store it, with the next plane's loads in
// flight.  The last NR threads (whole waves) stage the one-cell ring of
// densities around the tile and the n_s planes: they hold no collision state,
// so the cell waves keep their registers for the prefetch.
//
// LDS: four density / n_s plane slots (plane p in slot p mod 4, one barrier
// per plane) and the raw words of the last planes staged, private to each
// cell thread.  16-bit: two planes, and the collision reads its plane's words
// from LDS, so no register holds them while two planes of loads are in
// flight.  FP32: one plane (its words take twice the room), the plane being
// collided in registers, one plane of loads in flight.
template <typename ST, int CNS, int TX, int TY>
struct PairShared {
    using W = typename PairWordOf<ST>::W;
    static constexpr int LW = TX + 2;
    static constexpr int LP = LW * (TY + 2);
    static constexpr int NT = TX * TY;
    static constexpr int NB = sizeof(W) == 4 ? 2 : 1;  // planes of words held in LDS
    float rho[4][2][LP];
    float ns[4][CNS][LP];
    W hs[NB][kQ][NT];
};

constexpr int kPairRing = 192;  // ring / n_s threads per block (three waves)
#ifndef LBM_PAIR_TY
#define LBM_PAIR_TY 8
#endif
// Rows of the default pair tile (64 x kPairTY cells).  With eight rows the
// block has eight cell waves, an even share for each of a CU's four SIMDs (nine
// leave one SIMD a third collision per plane), and a 256 x 256 plane splits
// into 128 tile columns, so two z-chunks per column give one block for each of
// 256 CUs (nine rows: 116 columns, 232 blocks).
constexpr int kPairTY = LBM_PAIR_TY;

// Planes a cell wave keeps in flight ahead of the one it stages (1 or 2).
#ifndef LBM_PAIR_AHEAD
#define LBM_PAIR_AHEAD 2
#endif

// Rounding of the stored words: kRoundNearest and kRoundStochastic fix it at
// compile time; kRoundEither follows the domain's flag without a branch
// (both roundings computed and one selected), so that the stores of a
// collision form one straight sequence (after a branch between two store
// sequences the compiler's wait counts lose track of how many stores were
// issued, and its waits for the next plane's loads then wait for the
// stores as well).
constexpr int kRoundNearest = 0, kRoundStochastic = 1, kRoundEither = 2;

template <typename ST, int CNS, int TX, int TY, int FS, bool ONE, int RND>
__device__ __forceinline__ void step_tile_pair(const Args<float>& a,
                                               const typename PairWordOf<ST>::W* __restrict__ A,
                                               typename PairWordOf<ST>::W* __restrict__ B,
                                               const float* __restrict__ ns, int L, uint32_t t,
                                               PairShared<ST, CNS, TX, TY>& sh)
{
    using T = float;
    using W = typename PairWordOf<ST>::W;
    using PC = PairCodec<ST>;
    constexpr int LW = TX + 2;
    constexpr int LP = LW * (TY + 2);
    constexpr int NT = TX * TY;
    constexpr int NR = kPairRing;
    constexpr int NSR = (LP + NR - 1) / NR;  // n_s cells staged per ring thread and plane
    static_assert(NT % 64 == 0, "the roles must fill whole waves");
    static_assert(2 * (TX + 2) + 2 * TY <= NR, "one ring cell per ring thread");
    auto& s_rho = sh.rho;
    auto& s_ns = sh.ns;

    const int tx = L % a.ntx;
    const int ty = (L / a.ntx) % a.nty;
    const int tz = L / (a.ntx * a.nty);
    const int x0 = tx * TX, y0 = ty * TY;
    const int zs = tz * a.zchunk;
    const int ze = min(zs + a.zchunk, a.nz);
    const int TXe = min(TX, a.nx - x0);
    const int TYe = min(TY, a.ny - y0);
    const int plane = a.plane;
    const int tl = static_cast<int>(threadIdx.x);

    auto wrapz = [&](int p) { return p < 0 ? p + a.nz : (p >= a.nz ? p - a.nz : p); };
    // one buffer descriptor per plane block of 19 direction arrays of words
    const uint32_t dir_bytes = static_cast<uint32_t>(plane) * static_cast<uint32_t>(sizeof(W));
    const uint32_t blk_bytes = static_cast<uint32_t>(kQ) * dir_bytes;
    auto blk = [&](const W* base, int p) {
        return make_rsrc(base + static_cast<size_t>(p) * kQ * static_cast<size_t>(plane), blk_bytes);
    };
    auto issue = [&](int p, const PlaneOffs& q, W e[kQ]) {
        const rsrc_t r3[3] = {blk(A, wrapz(p + 1)), blk(A, p), blk(A, wrapz(p - 1))};  // c_z = -1, 0, +1
#pragma unroll
        for (int i = 0; i < kQ; ++i)
            e[i] = word_load<W>(r3[CZ[i] + 1], q.o[CY[i] + 1][CX[i] + 1], static_cast<uint32_t>(i) * dir_bytes);
    };
    // densities rho_0, rho_1 of a cell from its raw words, and with MOM its
    // first moments (Eq. mom_BGK) too; a reservoir cell has the Dirichlet
    // density instead, summed in the same order over the rest populations
    // w_i dr (computed only when a lane of the wave is in a reservoir), and
    // first moments 0 (w_i = w_ibar).  The words are decoded into the running
    // sums, never held as 38 floats.
    auto moments = [&](uint32_t rbits, const W e[kQ], T& r0, T& r1, T* j) {
        T s0 = PC::lo(e[0]), s1 = PC::hi(e[0]);
        T j0[3] = {T(0), T(0), T(0)}, j1[3] = {T(0), T(0), T(0)};
#pragma unroll
        for (int i = 1; i <= 9; ++i) {
            // sums and differences of opposite populations, each rounded once
            // (b - a is exactly -(a - b), so the sign goes into the update)
            const T p0 = PC::template sum<0>(e[i], e[i + 9]), p1 = PC::template sum<1>(e[i], e[i + 9]);
            s0 += p0;
            s1 += p1;
            if (j) {
                const T d0 = PC::template diff<0>(e[i], e[i + 9]), d1 = PC::template diff<1>(e[i], e[i + 9]);
                if (CX[i]) { j0[0] = CX[i] > 0 ? j0[0] + d0 : j0[0] - d0; j1[0] = CX[i] > 0 ? j1[0] + d1 : j1[0] - d1; }
                if (CY[i]) { j0[1] = CY[i] > 0 ? j0[1] + d0 : j0[1] - d0; j1[1] = CY[i] > 0 ? j1[1] + d1 : j1[1] - d1; }
                if (CZ[i]) { j0[2] = CZ[i] > 0 ? j0[2] + d0 : j0[2] - d0; j1[2] = CZ[i] > 0 ? j1[2] + d1 : j1[2] - d1; }
            }
        }
        s0 *= a.inv_scale;
        s1 *= a.inv_scale;
        if (j) {
            const bool in = rbits != 0;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                j[d] = in ? T(0) : j0[d] * a.inv_scale;
                j[3 + d] = in ? T(0) : j1[d] * a.inv_scale;
            }
        }
        const bool in = rbits != 0;
        if (__builtin_amdgcn_ballot_w64(in) != 0) {
            T dr0, dr1;
            reservoir_pick(a, rbits, dr0, dr1);
            T w0 = wgt<T>(0) * dr0, w1 = wgt<T>(0) * dr1;
#pragma unroll
            for (int i = 1; i <= 9; ++i) {
                w0 += wgt<T>(i) * dr0 + wgt<T>(i + 9) * dr0;
                w1 += wgt<T>(i) * dr1 + wgt<T>(i + 9) * dr1;
            }
            s0 = in ? w0 : s0;
            s1 = in ? w1 : s1;
        }
        r0 = a.rho0[0] + s0;
        r1 = a.rho0[1] + s1;
    };
    auto densities = [&](uint32_t rbits, const W e[kQ], T& r0, T& r1) {
        moments(rbits, e, r0, r1, static_cast<T*>(nullptr));
    };
    auto rslot = [&](int p) { return (p - zs + 1) & 3; };

    if (tl >= NT) {
        // ---- ring / n_s waves ----
        const int r = tl - NT;
        const int ring_n = 2 * (TXe + 2) + 2 * TYe;
        const bool ring = r < ring_n;
        int rlx, rly;
        {
            const int q = min(r, ring_n - 1);  // threads past the ring repeat its last cell
            if (q < TXe + 2) { rlx = q - 1; rly = -1; }
            else if (q < 2 * (TXe + 2)) { rlx = q - (TXe + 2) - 1; rly = TYe; }
            else if (q < 2 * (TXe + 2) + TYe) { rlx = -1; rly = q - 2 * (TXe + 2); }
            else { rlx = TXe; rly = q - 2 * (TXe + 2) - TYe; }
        }
        const int rx = ((x0 + rlx) % a.nx + a.nx) % a.nx;
        const int ry = ((y0 + rly) % a.ny + a.ny) % a.ny;
        const int rme = (rly + 1) * LW + (rlx + 1);
        const PlaneOffs qring = plane_offs<sizeof(W)>(rx, ry, a.nx, a.ny);
        const uint32_t rxy = reservoir_xy_bits(a, rx, ry);
        // n_s cells of this thread (LDS index, in-plane index); past the list
        // a thread repeats its first cell, the corner (x0 - 1, y0 - 1)
        const int nsw = TXe + 2, nsh = TYe + 2;
        const int ns_off0 = (((y0 - 1) % a.ny + a.ny) % a.ny) * a.nx + ((x0 - 1) % a.nx + a.nx) % a.nx;
        int nl[NSR], no[NSR];
#pragma unroll
        for (int k = 0; k < NSR; ++k) {
            const int c = r + k * NR;
            if (c < nsw * nsh) {
                const int llx = c % nsw - 1, lly = c / nsw - 1;
                const int gx = ((x0 + llx) % a.nx + a.nx) % a.nx;
                const int gy = ((y0 + lly) % a.ny + a.ny) % a.ny;
                nl[k] = (lly + 1) * LW + llx + 1;
                no[k] = gy * a.nx + gx;
            } else {
                nl[k] = 0;
                no[k] = ns_off0;
            }
        }
        W er[kQ];
        float nsv[NSR][CNS];
        auto issue_ring = [&](int p) {
            issue(p, qring, er);
            const float* nsp = ns + static_cast<size_t>(p) * static_cast<size_t>(plane);
#pragma unroll
            for (int k = 0; k < NSR; ++k)
#pragma unroll
                for (int c = 0; c < CNS; ++c) nsv[k][c] = nsp[static_cast<size_t>(c) * a.N + no[k]];
        };
        // consume the loads of plane p into LDS slot `slot`
        auto consume_ring = [&](int p, int slot) {
            T r0, r1;
            densities(rxy | reservoir_z_bits(a, p), er, r0, r1);
            if (ring) {
                s_rho[slot][0][rme] = r0;
                s_rho[slot][1][rme] = r1;
            }
#pragma unroll
            for (int k = 0; k < NSR; ++k)
#pragma unroll
                for (int c = 0; c < CNS; ++c) s_ns[slot][c][nl[k]] = nsv[k][c];
        };
        // ... then issue those of plane pn (unconditionally, so the waits stay
        // exact)
        auto stage_ring = [&](int p, int slot, int pn) {
            consume_ring(p, slot);
            __builtin_amdgcn_sched_barrier(0);
            issue_ring(pn);
        };
        if constexpr (ONE) {
            issue_ring(0);
            consume_ring(0, rslot(0));
            __syncthreads();
            return;
        } else {
            auto next = [&](int p) { return wrapz(p + 1 <= ze ? p + 1 : ze); };
            issue_ring(wrapz(zs - 1));
            stage_ring(wrapz(zs - 1), rslot(zs - 1), zs);
            stage_ring(zs, rslot(zs), next(zs));
            for (int z = zs; z < ze; ++z) {
                stage_ring(wrapz(z + 1), rslot(z + 1), next(z + 1));
                __syncthreads();
            }
            return;
        }
    }

    // ---- cell waves ----
    const int lx = tl % TX;
    const int ly = tl / TX;
    // a lane beyond a ragged tile edge duplicates the last active lane of its
    // row / column (same cell, same LDS slots, identical values written twice)
    const int x = x0 + min(lx, TXe - 1);
    const int y = y0 + min(ly, TYe - 1);
    const int me = (y - y0 + 1) * LW + (x - x0 + 1);
    const PlaneOffs qme = plane_offs<sizeof(W)>(x, y, a.nx, a.ny);
    const uint32_t own = static_cast<uint32_t>(y * a.nx + x) * static_cast<uint32_t>(sizeof(W));
    const uint32_t t_key = fmix32(t ^ kGolden);  // stochastic rounding: time part of the counter
    const uint32_t cxy = reservoir_xy_bits(a, x, y);

    // Collision of plane z from the raw words hz of the own cell and the LDS
    // slots of planes z-1, z, z+1.  The words are decoded where they are used
    // (twice: first moments, then the relaxation) rather than held as 38
    // floats.
    auto collide = [&](int z, int sm, int s0, int sp, const T (&jm)[6], auto&& wd) {
        const uint32_t rbits = cxy | reservoir_z_bits(a, z);
        const bool in = rbits != 0;
        T dr0, dr1;
        reservoir_pick(a, rbits, dr0, dr1);
        // populations on the stored scale: h_i * 2^k
        const T ds0 = dr0 * a.scale, ds1 = dr1 * a.scale;
        // (the word is read unconditionally: a conditional operator around
        // the read would become a branch per value)
        auto h0 = [&](int i) {
            const T v = PC::lo(wd(i));
            return in ? wgt<T>(i) * ds0 : v;
        };
        auto h1 = [&](int i) {
            const T v = PC::hi(wd(i));
            return in ? wgt<T>(i) * ds1 : v;
        };
        const T jc[2][3] = {{jm[0], jm[1], jm[2]}, {jm[3], jm[4], jm[5]}};
        T ueq[2][3], rho_own[2], n[2], fo[2][3];
        if constexpr (FS == kForcingGuo) {
            T um[3];
            cell_velocity_guo_pair<CNS, LW, LP>(a, me, &s_rho[sm][0][0], &s_rho[s0][0][0], &s_rho[sp][0][0],
                                                &s_ns[sm][0][0], &s_ns[s0][0][0], &s_ns[sp][0][0], jc, um, fo,
                                                rho_own, n);
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int d = 0; d < 3; ++d) ueq[c][d] = um[d];
        } else {
            cell_velocity_pair<CNS, LW, LP>(a, me, &s_rho[sm][0][0], &s_rho[s0][0][0], &s_rho[sp][0][0],
                                            &s_ns[sm][0][0], &s_ns[s0][0][0], &s_ns[sp][0][0], jc, ueq, rho_own, n);
        }
        RelaxCoef<T> k0 = relax_coef<T>(a, 0, rho_own[0], ueq[0], n[0]);
        RelaxCoef<T> k1 = relax_coef<T>(a, 1, rho_own[1], ueq[1], n[1]);
        GuoCoef<T> g0{}, g1{};
        if constexpr (FS == kForcingGuo) {
            g0 = guo_coef<T>(a, 0, n[0], fo[0], ueq[0]);
            g1 = guo_coef<T>(a, 1, n[1], fo[1], ueq[1]);
        }
        // the terms not proportional to h go to the stored scale
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            k0.K0[c] *= a.scale; k0.K1[c] *= a.scale; k0.K2[c] *= a.scale;
            k1.K0[c] *= a.scale; k1.K1[c] *= a.scale; k1.K2[c] *= a.scale;
            g0.gw[c] *= a.scale; g1.gw[c] *= a.scale;
        }
        auto rest = [&](const RelaxCoef<T>& k, const GuoCoef<T>& g, T h) {
            if constexpr (FS == kForcingGuo) return relax_rest_guo(k, g, h);
            else return relax_rest(k, h);
        };
        auto pairdir = [&](const RelaxCoef<T>& k, const GuoCoef<T>& g, int i, T hi_, T ho_, T& pi, T& po) {
            if constexpr (FS == kForcingGuo) relax_dir_guo(k, g, i, hi_, ho_, pi, po);
            else relax_dir(k, i, hi_, ho_, pi, po);
        };
        const rsrc_t rz = blk(B, z);
        // the random streams of the split kernels: per (cell, component)
        // fmix32 of the counter, then one lcg24 step per stored value
        uint32_t r0 = 0, r1 = 0;
        if constexpr (RND != kRoundNearest) {
            const uint32_t cell = static_cast<uint32_t>(z) * static_cast<uint32_t>(plane) + static_cast<uint32_t>(y * a.nx + x);
            r0 = fmix32(t_key ^ (2u * cell));
            r1 = fmix32(t_key ^ (2u * cell + 1u));
        }
        const uint32_t sr_mask = RND == kRoundEither ? 0u - static_cast<uint32_t>(a.sr != 0) : 0u;
        auto word = [&](T v0, T v1, uint32_t ra, uint32_t rb) -> W {
            if constexpr (RND == kRoundStochastic) return PC::enc_sr(v0, v1, ra, rb);
            else if constexpr (RND == kRoundNearest) return PC::enc(v0, v1);
            else return (PC::enc_sr(v0, v1, ra, rb) & sr_mask) | (PC::enc(v0, v1) & ~sr_mask);
        };
        word_store<W>(word(rest(k0, g0, h0(0)), rest(k1, g1, h1(0)), r0, r1), rz, own, 0u);
#pragma unroll
        for (int i = 1; i <= 9; ++i) {
            T pi0, po0, pi1, po1;
            pairdir(k0, g0, i, h0(i), h0(i + 9), pi0, po0);
            pairdir(k1, g1, i, h1(i), h1(i + 9), pi1, po1);
            uint32_t ri0 = 0, ri1 = 0;
            if constexpr (RND != kRoundNearest) {
                ri0 = lcg24(r0);
                ri1 = lcg24(r1);
                r0 = lcg24(ri0);
                r1 = lcg24(ri1);
            }
            word_store<W>(word(pi0, pi1, ri0, ri1), rz, own, static_cast<uint32_t>(i) * dir_bytes);
            word_store<W>(word(po0, po1, r0, r1), rz, own, static_cast<uint32_t>(i + 9) * dir_bytes);
        }
    };

    if constexpr (ONE) {
        // One cell deep: planes z - 1, z and z + 1 are all plane 0, staged
        // once and collided against itself.
        const int slot = rslot(0);
        W r1[kQ];
        issue(0, qme, r1);
        T d0, d1, jm[6];
        moments(cxy | reservoir_z_bits(a, 0), r1, d0, d1, jm);
        s_rho[slot][0][me] = d0;
        s_rho[slot][1][me] = d1;
        __syncthreads();
        collide(0, slot, slot, slot, jm, [&](int i) { return r1[i]; });
        return;
    } else if constexpr (sizeof(W) == 8) {
        // FP32 words: LDS holds one plane of them.  Plane z is collided from
        // registers (hz), plane z+1 waits in LDS (hs), and the loads of plane
        // z+2 are in flight over the barrier and the collision.  The ring
        // waves issue the ring loads of a plane at the same stage as these
        // own loads, while the neighbouring tiles' copies are still in L2.
        W* hsl = &sh.hs[0][0][0] + tl;
        W rc[kQ];
        W hz[kQ];
        T jA[6], jB[6];
        // Stage plane p, whose loads are in rc: densities to LDS, first
        // moments to jm, the words of the plane before from hs to hz and
        // plane p's into hs; then the loads of plane pn are issued.
        auto stage_pipe = [&](int p, int pu, int pn, T (&jm)[6]) {
            T d0, d1;
            moments(cxy | reservoir_z_bits(a, p), rc, d0, d1, jm);
            const int slot = rslot(pu);
            s_rho[slot][0][me] = d0;
            s_rho[slot][1][me] = d1;
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                hz[i] = hsl[i * NT];
                hsl[i * NT] = rc[i];
            }
            __builtin_amdgcn_sched_barrier(0);
            issue(pn, qme, rc);
        };
        auto wd = [&](int i) { return hz[i]; };
        // the plane whose loads a stage of plane p issues: p + 1, or after the
        // last plane the one just staged again (cache hits)
        auto next = [&](int p) { return wrapz(p + 1 <= ze ? p + 1 : ze); };
        issue(wrapz(zs - 1), qme, rc);
        stage_pipe(wrapz(zs - 1), zs - 1, zs, jB);
        stage_pipe(zs, zs, next(zs), jA);
        // unrolled by two so the moment sets keep fixed names
        for (int z = zs; z < ze; z += 2) {
            stage_pipe(wrapz(z + 1), z + 1, next(z + 1), jB);
            __syncthreads();
            collide(z, rslot(z - 1), rslot(z), rslot(z + 1), jA, wd);
            if (z + 1 >= ze) break;
            stage_pipe(wrapz(z + 2), z + 2, next(z + 2), jA);
            __syncthreads();
            collide(z + 1, rslot(z), rslot(z + 1), rslot(z + 2), jB, wd);
        }
    } else {
        // Three planes at a time: the words of planes z and z+1 wait in LDS
        // (hs, double-buffered), plane z is collided, and the loads of plane
        // z+1+AHEAD are in flight over the barrier and the collision.  No
        // memory access in the sweep is conditional (a skipped access would
        // make the compiler's waits drain the loads kept in flight).
        constexpr int AHEAD = LBM_PAIR_AHEAD;
        constexpr bool DEEP = AHEAD == 2;
        auto hbuf = [&](int p) { return &sh.hs[(p - zs + 2) & 1][0][0] + tl; };
        uint32_t rA[kQ];
        uint32_t rB[DEEP ? kQ : 1];
        // Stage plane p, whose loads are in rc: its densities go to LDS and
        // its words to hs; then the loads of plane pn are issued into rc.
        // the first moments of a staged plane wait in registers for its
        // collision (two sets, for the planes z and z+1)
        T jA[6], jB[6];
        auto stage_pipe = [&](int p, int pu, int pn, uint32_t rc[kQ], T (&jm)[6]) {
            T d0, d1;
            moments(cxy | reservoir_z_bits(a, p), rc, d0, d1, jm);
            const int slot = rslot(pu);
            s_rho[slot][0][me] = d0;
            s_rho[slot][1][me] = d1;
            uint32_t* hw = hbuf(pu);
#pragma unroll
            for (int i = 0; i < kQ; ++i) hw[i * NT] = rc[i];
            __builtin_amdgcn_sched_barrier(0);
            issue(pn, qme, rc);
        };
        auto collide_z = [&](int z, const T (&jm)[6]) {
            const uint32_t* hr = hbuf(z);
            collide(z, rslot(z - 1), rslot(z), rslot(z + 1), jm, [&](int i) { return hr[i * NT]; });
        };
        // the plane whose loads a stage of plane p issues: p + AHEAD, or after
        // the last plane one already staged again (cache hits)
        auto ahead = [&](int p) { return wrapz(p + AHEAD <= ze ? p + AHEAD : ze); };
        uint32_t (&r_odd)[kQ] = rA;
        uint32_t (&r_even)[kQ] = *reinterpret_cast<uint32_t(*)[kQ]>(DEEP ? static_cast<uint32_t*>(rB) : static_cast<uint32_t*>(rA));
        // prologue: planes zs-1 (densities only) and zs
        issue(wrapz(zs - 1), qme, r_odd);
        if constexpr (DEEP) issue(zs, qme, r_even);
        stage_pipe(wrapz(zs - 1), zs - 1, ahead(zs - 1), r_odd, jB);
        stage_pipe(zs, zs, ahead(zs), r_even, jA);
        // unrolled by two so the register sets keep fixed names
        for (int z = zs; z < ze; z += 2) {
            stage_pipe(wrapz(z + 1), z + 1, ahead(z + 1), r_odd, jB);
            __syncthreads();
            collide_z(z, jA);
            if (z + 1 >= ze) break;
            stage_pipe(wrapz(z + 2), z + 2, ahead(z + 2), r_even, jA);
            __syncthreads();
            collide_z(z + 1, jB);
        }
    }
}

// Two components in FP32 or a 16-bit format use the pair layout and kernel,
// except FP32 with the GS-WBS: its collision, with both components' Guo
// terms, needs more registers than the FP32 pair sweep leaves (it spilled and
// ran 4.6 % slower than in the split layout).
template <typename ST, int NC, int FS = kForcingShanChen>
constexpr bool kPair =
    (sizeof(typename ST::E) == 2 || (std::is_same_v<ST, F32> && FS != kForcingGuo)) && NC == 2;

template <typename ST, int NC, int TX, int TY, int FS = kForcingShanChen>
constexpr int kThreads = kPair<ST, NC, FS> ? TX * TY + kPairRing : NC * TX * TY;

template <typename ST, int NC, int CNS, int TX, int TY, int FS, bool ONE, int RND>
__global__ __launch_bounds__((kThreads<ST, NC, TX, TY, FS>)) void k_step(Args<typename ST::T> a,
                                                                    const typename ST::E* __restrict__ A,
                                                                    typename ST::E* __restrict__ B,
                                                                    const float* __restrict__ ns)
{
    // XCD-aware tile order: blocks are dispatched round-robin over 8 XCDs, so
    // give each XCD a contiguous run of tiles (neighbours share its L2).
    const int nb = gridDim.x;
    int L = blockIdx.x;
    if ((nb & 7) == 0) L = (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3);
    if constexpr (kPair<ST, NC, FS>) {
        using W = typename PairWordOf<ST>::W;
        __shared__ PairShared<ST, CNS, TX, TY> sh;
        step_tile_pair<ST, CNS, TX, TY, FS, ONE, RND>(a, reinterpret_cast<const W*>(A), reinterpret_cast<W*>(B), ns, L,
                                                      a.t, sh);
    } else {
        __shared__ TileShared<ST, NC, CNS, TX, TY> sh;
        step_tile<ST, NC, CNS, TX, TY, FS, ONE>(a, A, B, ns, L, a.t, sh);
    }
}

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
__global__ __launch_bounds__((kThreads<ST, NC, TX, TY>)) void k_step_batch(const char* __restrict__ table, int k)
{
    using T = typename ST::T;
    using E = typename ST::E;
    const BatchHeader* hdr = reinterpret_cast<const BatchHeader*>(table);
    const BatchEntry<T>* ent = reinterpret_cast<const BatchEntry<T>*>(table + kBatchEntryOffset);
    const int total = hdr->total_tiles;
    const int nd = hdr->ndom;
    // XCD-aware order, as in k_step: blocks are dispatched round-robin over
    // the 8 XCDs, so give each XCD a contiguous run of every stride of tiles
    // (neighbouring tiles re-read each other's edge cells through its L2)
    const int nb = gridDim.x;
    const int b0 = (nb & 7) == 0 ? (blockIdx.x & 7) * (nb >> 3) + (blockIdx.x >> 3) : blockIdx.x;
    using Shared = std::conditional_t<kPair<ST, NC>, PairShared<ST, CNS, TX, TY>, TileShared<ST, NC, CNS, TX, TY>>;
    __shared__ Shared sh;
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
        if constexpr (kPair<ST, NC>) {
            // the rounding of each domain picks a tile sweep compiled for it
            // (FP32 rounds to nearest only)
            using W = typename PairWordOf<ST>::W;
            const W* src = static_cast<const W*>(e.buf[cur]);
            W* dst = static_cast<W*>(const_cast<void*>(e.buf[1 - cur]));
            const uint32_t tk = e.a.t + static_cast<uint32_t>(k);
            constexpr int SR = sizeof(E) == 2 ? kRoundStochastic : kRoundNearest;
            if (e.a.sr)
                step_tile_pair<ST, CNS, TX, TY, kForcingShanChen, false, SR>(e.a, src, dst, e.ns, w - e.tile_begin,
                                                                             tk, sh);
            else
                step_tile_pair<ST, CNS, TX, TY, kForcingShanChen, false, kRoundNearest>(e.a, src, dst, e.ns,
                                                                                      w - e.tile_begin, tk, sh);
        } else
            step_tile<ST, NC, CNS, TX, TY, kForcingShanChen>(e.a, static_cast<const E*>(e.buf[cur]),
                                                             static_cast<E*>(const_cast<void*>(e.buf[1 - cur])), e.ns,
                                                             w - e.tile_begin, e.a.t + static_cast<uint32_t>(k), sh);
    }
}

// ---------------------------------------------------------------------------
// Auxiliary kernels (initialisation, checkpoints, FP64 diagnostics).  They run
// once per call, not per step: plain grid-stride loops over the cells.

#define CELL_LOOP(n, N)                                                                                      \
    for (int64_t n = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; n < (N);                  \
         n += static_cast<int64_t>(gridDim.x) * blockDim.x)

struct Cell {
    int x, y, z, ip;  // coordinates and in-plane index
};

template <typename T>
__device__ __forceinline__ Cell cell_of(const Args<T>& a, int64_t n)
{
    Cell c;
    c.z = static_cast<int>(n / a.plane);
    c.ip = static_cast<int>(n - static_cast<int64_t>(c.z) * a.plane);
    c.x = c.ip % a.nx;
    c.y = c.ip / a.nx;
    return c;
}

template <typename T>
__device__ __forceinline__ int64_t cell_at(const Args<T>& a, int x, int y, int z)
{
    return static_cast<int64_t>(z) * a.plane + y * a.nx + x;
}

// direction i as (cx, cy, cz, w_i) for a runtime i
template <typename T>
__device__ __forceinline__ void dir_of(int i, int& dx, int& dy, int& dz, T& w)
{
    dx = dy = dz = 0;
    w = T(0);
#pragma unroll
    for (int k = 0; k < kQ; ++k)
        if (k == i) {
            dx = CX[k];
            dy = CY[k];
            dz = CZ[k];
            w = wgt<T>(k);
        }
}

template <typename ST>
__global__ void k_init(Args<typename ST::T> a, int ncomp, const double* __restrict__ rho_init,
                       typename ST::E* __restrict__ A)
{
    using T = typename ST::T;
    CELL_LOOP(n, a.N)
    {
        const Cell c = cell_of(a, n);
        // A_i(y) must hold f_i(y + c_i, 0) (pull storage)
        for (int s = 0; s < ncomp; ++s) {
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const int xd = (c.x + CX[i] + a.nx) % a.nx, yd = (c.y + CY[i] + a.ny) % a.ny,
                          zd = (c.z + CZ[i] + a.nz) % a.nz;
                const int res = reservoir_of(a, xd, yd, zd);
                const double rho = res >= 0 ? static_cast<double>(a.res_dr[res][s]) + static_cast<double>(a.rho0[s])
                                            : rho_init[static_cast<size_t>(s) * a.N + cell_at(a, xd, yd, zd)];
                const double h = wgt<double>(i) * (rho - static_cast<double>(a.rho0[s]));
                A[pidx(a, s, i, c.z, c.ip)] = ST::enc(static_cast<T>(h), a.scale);
            }
        }
    }
}

template <typename ST>
__global__ void k_canonical(Args<typename ST::T> a, const typename ST::E* __restrict__ A, int s, int i,
                            double* __restrict__ out)
{
    int dx, dy, dz;
    double w;
    dir_of(i, dx, dy, dz, w);
    CELL_LOOP(n, a.N)
    {
        const Cell c = cell_of(a, n);
        const int res = reservoir_of(a, c.x, c.y, c.z);
        double v;
        if (res >= 0) {
            v = w * (static_cast<double>(a.res_dr[res][s]) + static_cast<double>(a.rho0[s]));
        } else {
            const int xs = (c.x - dx + a.nx) % a.nx, ys = (c.y - dy + a.ny) % a.ny, zs = (c.z - dz + a.nz) % a.nz;
            v = static_cast<double>(ST::dec(A[pidx(a, s, i, zs, ys * a.nx + xs)], a.inv_scale)) +
                w * static_cast<double>(a.rho0[s]);
        }
        out[n] = v;
    }
}

template <typename ST>
__global__ void k_set_canonical(Args<typename ST::T> a, const double* __restrict__ in, int s, int i,
                                typename ST::E* __restrict__ A)
{
    using T = typename ST::T;
    int dx, dy, dz;
    double w;
    dir_of(i, dx, dy, dz, w);
    CELL_LOOP(n, a.N)
    {
        const Cell c = cell_of(a, n);
        // A_i(y) = f_i(y + c_i)
        const int xd = (c.x + dx + a.nx) % a.nx, yd = (c.y + dy + a.ny) % a.ny, zd = (c.z + dz + a.nz) % a.nz;
        const double h = in[cell_at(a, xd, yd, zd)] - w * static_cast<double>(a.rho0[s]);
        A[pidx(a, s, i, c.z, c.ip)] = ST::enc(static_cast<T>(h), a.scale);
    }
}

constexpr int kRedThreads = 256;

// Sum of v over the block, the same on every run: a butterfly over each
// wave's 64 lanes (cross-lane moves, no LDS round trips or barriers), then
// the waves' sums in wave order; thread k < K writes out[k].
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* __restrict__ out)
{
    __shared__ double ws[kRedThreads / 64][K];
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    const int wv = static_cast<int>(threadIdx.x) >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) ws[wv][k] = v[k];
    __syncthreads();
    if (threadIdx.x < K) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kRedThreads / 64; ++w) s += ws[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

// Diagnostics, first pass (the only one that reads the populations): per cell
// the FP64 densities rho_s (Eq. rho_BGK) and first moments j_s (Eq. mom_BGK) of
// the pre-collision state; writes rho [ncomp][N] and, when m_out is given, the
// local part of rho u_macro of Eq. (HMCSC_u_macro), sum_s (1 - n_s)(j_s +
// F_ext,s / 2) with F_ext,s of Eq. (SC_F_ext), into m_out [3][N].  Block
// totals {M_0, M_1, sum of that local part} go to partials[block][5].
template <typename ST>
__global__ __launch_bounds__(kRedThreads) void k_dens(Args<typename ST::T> a, int ncomp, int c_ns,
                                                      const typename ST::E* __restrict__ A,
                                                      const float* __restrict__ ns, double* __restrict__ rho,
                                                      double* __restrict__ m_out, double* __restrict__ partials)
{
    double acc[5] = {0, 0, 0, 0, 0};
    CELL_LOOP(n, a.N)
    {
        const Cell c = cell_of(a, n);
        const int res = reservoir_of(a, c.x, c.y, c.z);
        const int xs[3] = {wrap_inc(c.x, a.nx), c.x, wrap_dec(c.x, a.nx)};  // x - c, c = -1, 0, 1
        const int ys[3] = {wrap_inc(c.y, a.ny), c.y, wrap_dec(c.y, a.ny)};
        const int zs[3] = {wrap_inc(c.z, a.nz), c.z, wrap_dec(c.z, a.nz)};
        double rs[2] = {0, 0}, j[2][3] = {{0, 0, 0}, {0, 0, 0}}, rtot = 0;
        for (int s = 0; s < ncomp; ++s) {
            double d = 0;
            if (res >= 0) {
                d = static_cast<double>(a.res_dr[res][s]);
            } else {
#pragma unroll
                for (int i = 0; i < kQ; ++i) {
                    const double h = static_cast<double>(
                        ST::dec(A[pidx(a, s, i, zs[CZ[i] + 1], ys[CY[i] + 1] * a.nx + xs[CX[i] + 1])], a.inv_scale));
                    d += h;
                    j[s][0] += CX[i] * h;
                    j[s][1] += CY[i] * h;
                    j[s][2] += CZ[i] * h;
                }
            }
            rs[s] = static_cast<double>(a.rho0[s]) + d;
            rho[static_cast<size_t>(s) * a.N + n] = rs[s];
            rtot += rs[s];
        }
        double m[3] = {0, 0, 0};
        for (int s = 0; s < ncomp; ++s) {
            const double wfl = 1.0 - static_cast<double>(ns[static_cast<size_t>(c_ns == 2 ? s : 0) * a.N + n]);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double fext = rtot > 0 ? rs[s] / rtot * static_cast<double>(a.F[d]) : 0.0;
                m[d] += wfl * (j[s][d] + fext / 2.0);
            }
        }
        if (m_out)
#pragma unroll
            for (int d = 0; d < 3; ++d) m_out[static_cast<size_t>(d) * a.N + n] = m[d];
        acc[0] += rs[0];
        acc[1] += rs[1];
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[2 + d] += m[d];
    }
    block_sum<5>(acc, partials + static_cast<size_t>(blockIdx.x) * 5);
}

// Diagnostics, second pass (densities and n_s only): the half cohesion and
// adhesion forces of Eqs. (SC_F_inter), (SC_F_ads) weighted by (1 - n_s), the
// rest of rho u_macro.  When u is given it holds the first pass's local part
// and receives u_macro of Eq. (HMCSC_u_macro); p receives Eq. (SC_pressure).
// Block totals {0, 0, sum of the force part} go to partials[block][5].
template <typename T>
__global__ __launch_bounds__(kRedThreads) void k_force(Args<T> a, int ncomp, int c_ns, double G_s, double Gads0,
                                                       double Gads1, double gG_p, const float* __restrict__ ns,
                                                       const double* __restrict__ rho, double* __restrict__ u,
                                                       double* __restrict__ p_out, double* __restrict__ partials)
{
    double acc[5] = {0, 0, 0, 0, 0};
    const double Gads[2] = {Gads0, Gads1};
    CELL_LOOP(n, a.N)
    {
        const Cell c = cell_of(a, n);
        // neighbours x + c_i (note: opposite of the pull)
        const int cols[3] = {wrap_dec(c.x, a.nx), c.x, wrap_inc(c.x, a.nx)};
        const int rows[3] = {wrap_dec(c.y, a.ny), c.y, wrap_inc(c.y, a.ny)};
        const int plns[3] = {wrap_dec(c.z, a.nz), c.z, wrap_inc(c.z, a.nz)};
        double rs[2] = {0, 0}, rtot = 0;
        for (int s = 0; s < ncomp; ++s) {
            rs[s] = rho[static_cast<size_t>(s) * a.N + n];
            rtot += rs[s];
        }
        double m[3] = {0, 0, 0};
        for (int s = 0; s < ncomp; ++s) {
            double gi[3] = {0, 0, 0}, ga[3] = {0, 0, 0};
            const size_t cn = static_cast<size_t>(c_ns == 2 ? s : 0);
#pragma unroll
            for (int i = 1; i < kQ; ++i) {
                const int64_t nb = cell_at(a, cols[CX[i] + 1], rows[CY[i] + 1], plns[CZ[i] + 1]);
                const double wi = wgt<double>(i);
                if (ncomp == 2) {
                    const double r = rho[static_cast<size_t>(1 - s) * a.N + nb];
                    gi[0] += wi * r * CX[i]; gi[1] += wi * r * CY[i]; gi[2] += wi * r * CZ[i];
                }
                const double v = static_cast<double>(ns[cn * a.N + nb]);
                ga[0] += wi * v * CX[i]; ga[1] += wi * v * CY[i]; ga[2] += wi * v * CZ[i];
            }
            const double wfl = 1.0 - static_cast<double>(ns[cn * a.N + n]);
#pragma unroll
            for (int d = 0; d < 3; ++d) m[d] += wfl * ((-rs[s] * G_s * gi[d] - rs[s] * Gads[s] * ga[d]) / 2.0);
        }
        if (u)
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                double& ud = u[static_cast<size_t>(d) * a.N + n];
                ud = rtot > 0 ? (ud + m[d]) / rtot : 0.0;
            }
        if (p_out) p_out[n] = (rtot + (ncomp == 2 ? gG_p * rs[0] * rs[1] : 0.0)) / 3.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[2 + d] += m[d];
    }
    block_sum<5>(acc, partials + static_cast<size_t>(blockIdx.x) * 5);
}

// FP64 density of component s at cell (x, y, z) of the pre-collision state:
// the pulled populations summed in direction order, or the reservoir's
// prescribed density.
template <typename ST>
__device__ __forceinline__ double density_at(const Args<typename ST::T>& a, const typename ST::E* __restrict__ A,
                                             int s, int x, int y, int z)
{
    const int res = reservoir_of(a, x, y, z);
    double d = 0;
    if (res >= 0) {
        d = static_cast<double>(a.res_dr[res][s]);
    } else {
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int xs = (x - CX[i] + a.nx) % a.nx, ys = (y - CY[i] + a.ny) % a.ny, zs = (z - CZ[i] + a.nz) % a.nz;
            d += static_cast<double>(ST::dec(A[pidx(a, s, i, zs, ys * a.nx + xs)], a.inv_scale));
        }
    }
    return static_cast<double>(a.rho0[s]) + d;
}

// The FP64 totals of k_dens and k_force in one pass with no per-cell field:
// each cell recomputes the densities of its 18 neighbours from their pulled
// populations (19 times the reads of one pass, cache hits for the most part).
// Block totals {M_0, M_1, J_x, J_y, J_z} go to partials[block][5].
template <typename ST>
__global__ __launch_bounds__(kRedThreads) void k_totals_one_pass(Args<typename ST::T> a, int ncomp, int c_ns,
                                                                 double G_s, double Gads0, double Gads1,
                                                                 const typename ST::E* __restrict__ A,
                                                                 const float* __restrict__ ns,
                                                                 double* __restrict__ partials)
{
    double acc[5] = {0, 0, 0, 0, 0};
    const double Gads[2] = {Gads0, Gads1};
    CELL_LOOP(n, a.N)
    {
        const Cell c = cell_of(a, n);
        const int res = reservoir_of(a, c.x, c.y, c.z);
        const int xs[3] = {wrap_inc(c.x, a.nx), c.x, wrap_dec(c.x, a.nx)};  // x - c, c = -1, 0, 1
        const int ys[3] = {wrap_inc(c.y, a.ny), c.y, wrap_dec(c.y, a.ny)};
        const int zs[3] = {wrap_inc(c.z, a.nz), c.z, wrap_dec(c.z, a.nz)};
        double rs[2] = {0, 0}, j[2][3] = {{0, 0, 0}, {0, 0, 0}}, rtot = 0;
        for (int s = 0; s < ncomp; ++s) {
            if (res < 0) {
#pragma unroll
                for (int i = 0; i < kQ; ++i) {
                    const double h = static_cast<double>(
                        ST::dec(A[pidx(a, s, i, zs[CZ[i] + 1], ys[CY[i] + 1] * a.nx + xs[CX[i] + 1])], a.inv_scale));
                    j[s][0] += CX[i] * h;
                    j[s][1] += CY[i] * h;
                    j[s][2] += CZ[i] * h;
                }
            }
            rs[s] = density_at<ST>(a, A, s, c.x, c.y, c.z);
            rtot += rs[s];
        }
        double m[3] = {0, 0, 0};
        for (int s = 0; s < ncomp; ++s) {
            double gi[3] = {0, 0, 0}, ga[3] = {0, 0, 0};
            const size_t cn = static_cast<size_t>(c_ns == 2 ? s : 0);
#pragma unroll
            for (int i = 1; i < kQ; ++i) {
                // neighbour x + c_i
                const int nx_ = (c.x + CX[i] + a.nx) % a.nx, ny_ = (c.y + CY[i] + a.ny) % a.ny,
                          nz_ = (c.z + CZ[i] + a.nz) % a.nz;
                const double wi = wgt<double>(i);
                if (ncomp == 2) {
                    const double r = density_at<ST>(a, A, 1 - s, nx_, ny_, nz_);
                    gi[0] += wi * r * CX[i]; gi[1] += wi * r * CY[i]; gi[2] += wi * r * CZ[i];
                }
                const double v = static_cast<double>(ns[cn * a.N + cell_at(a, nx_, ny_, nz_)]);
                ga[0] += wi * v * CX[i]; ga[1] += wi * v * CY[i]; ga[2] += wi * v * CZ[i];
            }
            const double wfl = 1.0 - static_cast<double>(ns[cn * a.N + n]);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double fext = rtot > 0 ? rs[s] / rtot * static_cast<double>(a.F[d]) : 0.0;
                const double ft = -rs[s] * G_s * gi[d] - rs[s] * Gads[s] * ga[d] + fext;
                m[d] += wfl * (j[s][d] + ft / 2.0);
            }
        }
        acc[0] += rs[0];
        acc[1] += rs[1];
#pragma unroll
        for (int d = 0; d < 3; ++d) acc[2 + d] += m[d];
    }
    block_sum<5>(acc, partials + static_cast<size_t>(blockIdx.x) * 5);
}

// Electrolyte-filling diagnostics (Sec. 4) from the FP64 fields: per-block
// sums of p and cell counts over the inlet and outlet slabs (Eq. CapPressure),
// and of (1 - n_s) [rho_comp >= threshold] and (1 - n_s) over the pore slab
// (Eq. Saturation).
__global__ __launch_bounds__(kRedThreads) void k_fill(int nx, int ny, int nz, int64_t N, FillQuery q, int ns_field,
                                                      const double* __restrict__ rho, const double* __restrict__ p,
                                                      const float* __restrict__ ns, double* __restrict__ partials)
{
    double acc[6] = {0, 0, 0, 0, 0, 0};
    const int64_t plane = static_cast<int64_t>(nx) * ny;
    CELL_LOOP(n, N)
    {
        const int z = static_cast<int>(n / plane);
        const int ip = static_cast<int>(n - z * plane);
        const int x = ip % nx, y = ip / nx;
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
    (void)nz;
    block_sum<6>(acc, partials + static_cast<size_t>(blockIdx.x) * 6);
}

// Permeability (Eq. Permeability) from the FP64 fields: per-block sums of
// rho_s u_macro[axis] for each component (the component's share of the
// mixture momentum, used for relative permeabilities) and of rho u_macro[axis].
__global__ __launch_bounds__(kRedThreads) void k_flux(int64_t N, int ncomp, int axis, const double* __restrict__ rho,
                                                      const double* __restrict__ u, double* __restrict__ partials)
{
    double acc[3] = {0, 0, 0};
    CELL_LOOP(n, N)
    {
        const double ua = u[static_cast<size_t>(axis) * N + n];
        const double r0 = rho[n];
        const double r1 = ncomp == 2 ? rho[static_cast<size_t>(N) + n] : 0.0;
        acc[0] += r0 * ua;
        acc[1] += r1 * ua;
        acc[2] += (r0 + r1) * ua;
    }
    block_sum<3>(acc, partials + static_cast<size_t>(blockIdx.x) * 3);
}

// Static-droplet measurement (Sec. 3.3) from an FP64 field f: per-block sums
// of f and cell counts over the ball |x - c| <= sqrt(r_in2) and over the
// cells with |x - c| >= sqrt(r_out2), distances taken to the nearest periodic
// image of the centre c (2-D when nz = 1).
__global__ __launch_bounds__(kRedThreads) void k_ball(int nx, int ny, int nz, int64_t N, double cx, double cy,
                                                      double cz, double r_in2, double r_out2,
                                                      const double* __restrict__ f, double* __restrict__ partials)
{
    double acc[4] = {0, 0, 0, 0};
    const int64_t plane = static_cast<int64_t>(nx) * ny;
    CELL_LOOP(n, N)
    {
        const int z = static_cast<int>(n / plane);
        const int ip = static_cast<int>(n - z * plane);
        const int x = ip % nx, y = ip / nx;
        double dx = x - cx, dy = y - cy, dz = z - cz;
        dx -= nx * rint(dx / nx);
        dy -= ny * rint(dy / ny);
        dz -= nz * rint(dz / nz);
        const double d2 = dx * dx + dy * dy + dz * dz;
        if (d2 <= r_in2) {
            acc[0] += f[n];
            acc[1] += 1.0;
        }
        if (d2 >= r_out2) {
            acc[2] += f[n];
            acc[3] += 1.0;
        }
    }
    block_sum<4>(acc, partials + static_cast<size_t>(blockIdx.x) * 4);
}

// Fixed-order sum of nblocks partials of K doubles each (one block): the
// result does not depend on timing.
template <int K>
__global__ __launch_bounds__(kRedThreads) void k_reduce(const double* __restrict__ partials, int nblocks,
                                                        double* __restrict__ out)
{
    double acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kRedThreads)
#pragma unroll
        for (int k = 0; k < K; ++k) acc[k] += partials[static_cast<size_t>(b) * K + k];
    block_sum<K>(acc, out);
}

// ---------------------------------------------------------------------------
// Launchers.

bool pair_layout(int storage, int ncomp, int forcing)
{
    return ((storage == kF32 && forcing != kForcingGuo) || storage == kF16 || storage == kBF16) && ncomp == 2;
}

int pair_tile_y() { return kPairTY; }

bool tile_supported(int storage, int ncomp, int tx, int ty, int forcing)
{
    if (pair_layout(storage, ncomp, forcing)) return tx == 64 && (ty == kPairTY || ty == 4);
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
    // the pair kernel is compiled per rounding mode; the split kernels
    // branch on it (their two store sequences are alike)
    if constexpr (kPair<ST, NC, FS>) {
        constexpr int SR = sizeof(E) == 2 ? kRoundStochastic : kRoundNearest;  // FP32 rounds to nearest
        if (p.stochastic)
            hipLaunchKernelGGL((k_step<ST, NC, CNS, TX, TY, FS, ONE, SR>), dim3(nblocks),
                               dim3(kThreads<ST, NC, TX, TY, FS>), 0, st, a, static_cast<const E*>(A),
                               static_cast<E*>(B), ns);
        else
            hipLaunchKernelGGL((k_step<ST, NC, CNS, TX, TY, FS, ONE, kRoundNearest>), dim3(nblocks),
                               dim3(kThreads<ST, NC, TX, TY, FS>), 0, st, a, static_cast<const E*>(A),
                               static_cast<E*>(B), ns);
    } else {
        hipLaunchKernelGGL((k_step<ST, NC, CNS, TX, TY, FS, ONE, kRoundEither>), dim3(nblocks),
                           dim3(kThreads<ST, NC, TX, TY, FS>), 0, st, a, static_cast<const E*>(A), static_cast<E*>(B),
                           ns);
    }
    return hipGetLastError();
}

// The default tiles of a layout, with the one-plane and GS-WBS instances.
template <typename ST, int NC, int CNS, int TX, int TY>
static hipError_t step_default(const Problem& p, const Launch& l, int64_t t, const void* A, void* B, const float* ns,
                               hipStream_t st)
{
    constexpr int SC = kForcingShanChen, GUO = kForcingGuo;
    const bool one = p.nz == 1;
    if (p.forcing == kForcingGuo)
        return one ? step_t<ST, NC, CNS, TX, TY, GUO, true>(p, l, t, A, B, ns, st)
                   : step_t<ST, NC, CNS, TX, TY, GUO, false>(p, l, t, A, B, ns, st);
    return one ? step_t<ST, NC, CNS, TX, TY, SC, true>(p, l, t, A, B, ns, st)
               : step_t<ST, NC, CNS, TX, TY, SC, false>(p, l, t, A, B, ns, st);
}

// Tile shapes (TX x TY cells per block) compiled in.
template <typename ST, int NC, int CNS>
static hipError_t step_ty(const Problem& p, const Launch& l, int64_t t, const void* A, void* B, const float* ns,
                          hipStream_t st)
{
    constexpr int SC = kForcingShanChen;
    if constexpr (kPair<ST, NC>) {
        if (l.tile_x == 64 && l.tile_y == kPairTY) return step_default<ST, NC, CNS, 64, kPairTY>(p, l, t, A, B, ns, st);
        if (l.tile_x == 64 && l.tile_y == 4) return step_default<ST, NC, CNS, 64, 4>(p, l, t, A, B, ns, st);
        return hipErrorInvalidValue;
    } else {
        if (l.tile_x == 64 && l.tile_y == 8) return step_default<ST, NC, CNS, 64, 8>(p, l, t, A, B, ns, st);
        if (l.tile_x == 64 && l.tile_y == 4) return step_default<ST, NC, CNS, 64, 4>(p, l, t, A, B, ns, st);
        if (p.forcing == kForcingGuo || p.nz == 1) return hipErrorInvalidValue;  // default tiles only
        if (l.tile_x == 128 && l.tile_y == 4) return step_t<ST, NC, CNS, 128, 4, SC, false>(p, l, t, A, B, ns, st);
        if (l.tile_x == 32 && l.tile_y == 4) return step_t<ST, NC, CNS, 32, 4, SC, false>(p, l, t, A, B, ns, st);
        if (l.tile_x == 32 && l.tile_y == 8) return step_t<ST, NC, CNS, 32, 8, SC, false>(p, l, t, A, B, ns, st);
        if (l.tile_x == 32 && l.tile_y == 16) return step_t<ST, NC, CNS, 32, 16, SC, false>(p, l, t, A, B, ns, st);
        return hipErrorInvalidValue;
    }
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

// Grid of a cell loop: enough blocks to fill the device a few times over.
static unsigned cell_blocks(int64_t N)
{
    return static_cast<unsigned>(std::min<int64_t>((N + 255) / 256, int64_t(1) << 20));
}

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

int moments_max_blocks() { return 1024; }

static int diag_blocks(int64_t N)
{
    return static_cast<int>(std::min<int64_t>(moments_max_blocks(), (N + kRedThreads - 1) / kRedThreads));
}

hipError_t launch_diagnostics(const Problem& p, const void* A, const float* ns, bool forces, double* rho, double* u,
                              double* pr, double* partials, double* out, hipStream_t st)
{
    const int nb = diag_blocks(p.N);
    hipError_t e = by_storage(p.storage, [&](auto tag) {
        using ST = decltype(tag);
        Args<typename ST::T> a = make_args<typename ST::T>(p);
        hipLaunchKernelGGL((k_dens<ST>), dim3(nb), dim3(kRedThreads), 0, st, a, p.ncomp, p.c_ns,
                           static_cast<const typename ST::E*>(A), ns, rho, u, partials);
        if (forces)
            hipLaunchKernelGGL((k_force<typename ST::T>), dim3(nb), dim3(kRedThreads), 0, st, a, p.ncomp, p.c_ns, p.G_s,
                               p.Gads_s[0], p.Gads_s[1], p.g_scale * p.G_inter, ns, rho, u, pr,
                               partials + static_cast<size_t>(nb) * 5);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce<5>, dim3(1), dim3(kRedThreads), 0, st, partials, forces ? 2 * nb : nb, out);
    return hipGetLastError();
}

hipError_t launch_totals_one_pass(const Problem& p, const void* A, const float* ns, double* partials, int max_blocks,
                                  double* out, hipStream_t st)
{
    const int nb = static_cast<int>(std::min<int64_t>(max_blocks, (p.N + kRedThreads - 1) / kRedThreads));
    hipError_t e = by_storage(p.storage, [&](auto tag) {
        using ST = decltype(tag);
        Args<typename ST::T> a = make_args<typename ST::T>(p);
        hipLaunchKernelGGL((k_totals_one_pass<ST>), dim3(nb), dim3(kRedThreads), 0, st, a, p.ncomp, p.c_ns, p.G_s,
                           p.Gads_s[0], p.Gads_s[1], static_cast<const typename ST::E*>(A), ns, partials);
        return hipGetLastError();
    });
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce<5>, dim3(1), dim3(kRedThreads), 0, st, partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_fill(const Problem& p, const FillQuery& q, const double* rho, const double* pr, const float* ns,
                       double* partials, double* out, hipStream_t st)
{
    const int nb = diag_blocks(p.N);
    const int ns_field = p.c_ns == 2 ? q.comp : 0;
    hipLaunchKernelGGL(k_fill, dim3(nb), dim3(kRedThreads), 0, st, p.nx, p.ny, p.nz, p.N, q, ns_field, rho, pr, ns,
                       partials);
    hipLaunchKernelGGL(k_reduce<6>, dim3(1), dim3(kRedThreads), 0, st, partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_ball(const Problem& p, const double c[3], double r_in, double r_out, const double* f,
                       double* partials, double* out, hipStream_t st)
{
    const int nb = diag_blocks(p.N);
    hipLaunchKernelGGL(k_ball, dim3(nb), dim3(kRedThreads), 0, st, p.nx, p.ny, p.nz, p.N, c[0], c[1], c[2],
                       r_in * r_in, r_out * r_out, f, partials);
    hipLaunchKernelGGL(k_reduce<4>, dim3(1), dim3(kRedThreads), 0, st, partials, nb, out);
    return hipGetLastError();
}

hipError_t launch_flux(const Problem& p, int axis, const double* rho, const double* u, double* partials, double* out,
                       hipStream_t st)
{
    const int nb = diag_blocks(p.N);
    hipLaunchKernelGGL(k_flux, dim3(nb), dim3(kRedThreads), 0, st, p.N, p.ncomp, axis, rho, u, partials);
    hipLaunchKernelGGL(k_reduce<3>, dim3(1), dim3(kRedThreads), 0, st, partials, nb, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Convergence monitor of the server: for every domain of a table, the FP64
// sums over its cells of the local part of rho u_macro (Eq. HMCSC_u_macro
// without the neighbour forces), sum_s (1 - n_s)(j_s + F_ext,s / 2), and of
// the mass.  One launch covers all domains (each owns a run of blocks); a
// second launch reduces each domain's blocks in a fixed order.
template <typename T>
struct MonitorEntry {
    Args<T> a;
    const void* state;
    const float* ns;
    int ncomp, c_ns;
    int block_begin, nblocks;
};

struct MonitorHeader {
    int ndom;
    int total_blocks;
    int pad[2];
};

template <typename ST>
__global__ __launch_bounds__(kRedThreads) void k_monitor(const char* __restrict__ table, double* __restrict__ partials)
{
    using T = typename ST::T;
    const MonitorHeader* hdr = reinterpret_cast<const MonitorHeader*>(table);
    const MonitorEntry<T>* ent = reinterpret_cast<const MonitorEntry<T>*>(table + kBatchEntryOffset);
    const int b = blockIdx.x;
    int lo = 0, hi = hdr->ndom - 1;  // last domain with block_begin <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ent[mid].block_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    const MonitorEntry<T>& e = ent[lo];
    const Args<T>& a = e.a;
    const typename ST::E* A = static_cast<const typename ST::E*>(e.state);
    double acc[4] = {0, 0, 0, 0};
    const int64_t stride = static_cast<int64_t>(e.nblocks) * blockDim.x;
    for (int64_t n = static_cast<int64_t>(b - e.block_begin) * blockDim.x + threadIdx.x; n < a.N; n += stride) {
        const Cell c = cell_of(a, n);
        const int res = reservoir_of(a, c.x, c.y, c.z);
        const int xs[3] = {wrap_inc(c.x, a.nx), c.x, wrap_dec(c.x, a.nx)};
        const int ys[3] = {wrap_inc(c.y, a.ny), c.y, wrap_dec(c.y, a.ny)};
        const int zs[3] = {wrap_inc(c.z, a.nz), c.z, wrap_dec(c.z, a.nz)};
        double rs[2] = {0, 0}, j[2][3] = {{0, 0, 0}, {0, 0, 0}}, rtot = 0;
        for (int s = 0; s < e.ncomp; ++s) {
            double d = 0;
            if (res >= 0) {
                d = static_cast<double>(a.res_dr[res][s]);
            } else {
#pragma unroll
                for (int i = 0; i < kQ; ++i) {
                    const double h = static_cast<double>(
                        ST::dec(A[pidx(a, s, i, zs[CZ[i] + 1], ys[CY[i] + 1] * a.nx + xs[CX[i] + 1])], a.inv_scale));
                    d += h;
                    j[s][0] += CX[i] * h;
                    j[s][1] += CY[i] * h;
                    j[s][2] += CZ[i] * h;
                }
            }
            rs[s] = static_cast<double>(a.rho0[s]) + d;
            rtot += rs[s];
        }
        for (int s = 0; s < e.ncomp; ++s) {
            const double wfl = 1.0 - static_cast<double>(e.ns[static_cast<size_t>(e.c_ns == 2 ? s : 0) * a.N + n]);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double fext = rtot > 0 ? rs[s] / rtot * static_cast<double>(a.F[d]) : 0.0;
                acc[d] += wfl * (j[s][d] + fext / 2.0);
            }
        }
        acc[3] += rtot;
    }
    block_sum<4>(acc, partials + static_cast<size_t>(b) * 4);
}

template <typename ST>
__global__ __launch_bounds__(kRedThreads) void k_monitor_reduce(const char* __restrict__ table,
                                                                const double* __restrict__ partials,
                                                                double* __restrict__ out)
{
    using T = typename ST::T;
    const MonitorEntry<T>* ent = reinterpret_cast<const MonitorEntry<T>*>(table + kBatchEntryOffset);
    const MonitorEntry<T>& e = ent[blockIdx.x];
    double acc[4] = {0, 0, 0, 0};
    for (int b = threadIdx.x; b < e.nblocks; b += kRedThreads)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += partials[static_cast<size_t>(e.block_begin + b) * 4 + k];
    block_sum<4>(acc, out + static_cast<size_t>(blockIdx.x) * 4);
}

template <typename T>
static size_t monitor_bytes_t(int max_domains)
{
    return kBatchEntryOffset + sizeof(MonitorEntry<T>) * static_cast<size_t>(max_domains > 0 ? max_domains : 1);
}

size_t monitor_table_bytes(int storage, int max_domains)
{
    return storage == kF64 ? monitor_bytes_t<double>(max_domains) : monitor_bytes_t<float>(max_domains);
}

int monitor_max_blocks(int max_domains) { return kMonitorBlocksPerDomain * (max_domains > 0 ? max_domains : 1); }

template <typename T>
static int monitor_encode_t(const MonitorDomain* d, int n, void* host)
{
    MonitorHeader* h = static_cast<MonitorHeader*>(host);
    MonitorEntry<T>* e = reinterpret_cast<MonitorEntry<T>*>(static_cast<char*>(host) + kBatchEntryOffset);
    int blocks = 0;
    for (int i = 0; i < n; ++i) {
        e[i].a = make_args<T>(d[i].prob);
        e[i].state = d[i].state;
        e[i].ns = d[i].ns;
        e[i].ncomp = d[i].prob.ncomp;
        e[i].c_ns = d[i].prob.c_ns;
        e[i].block_begin = blocks;
        e[i].nblocks = static_cast<int>(
            std::max<int64_t>(1, std::min<int64_t>(kMonitorBlocksPerDomain, (d[i].prob.N + 4095) / 4096)));
        blocks += e[i].nblocks;
    }
    h->ndom = n;
    h->total_blocks = blocks;
    h->pad[0] = h->pad[1] = 0;
    return blocks;
}

int monitor_encode(int storage, const MonitorDomain* d, int n, void* host)
{
    return storage == kF64 ? monitor_encode_t<double>(d, n, host) : monitor_encode_t<float>(d, n, host);
}

hipError_t launch_monitor(int storage, const void* table, int ndom, int total_blocks, double* partials, double* out,
                          hipStream_t st)
{
    if (ndom < 1) return hipSuccess;
    return by_storage(storage, [&](auto tag) {
        using ST = decltype(tag);
        hipLaunchKernelGGL((k_monitor<ST>), dim3(total_blocks), dim3(kRedThreads), 0, st,
                           static_cast<const char*>(table), partials);
        hipLaunchKernelGGL((k_monitor_reduce<ST>), dim3(ndom), dim3(kRedThreads), 0, st,
                           static_cast<const char*>(table), partials, out);
        return hipGetLastError();
    });
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
    hipLaunchKernelGGL((k_step_batch<ST, NC, CNS, TX, TY>), dim3(grid), dim3(kThreads<ST, NC, TX, TY>), 0, st,
                       static_cast<const char*>(table), k);
    return hipGetLastError();
}

template <typename ST, int NC, int CNS, int TX, int TY>
static int batch_occ_t()
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_batch<ST, NC, CNS, TX, TY>, kThreads<ST, NC, TX, TY>,
                                                     0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

// One function for every (format, components, n_s fields, tile) of the
// batched kernel: f receives the compiled instance's launcher and occupancy.
template <typename ST, int NC, int CNS, typename F>
static hipError_t batch_tile(int tx, int ty, F&& f)
{
    if constexpr (kPair<ST, NC>) {
        if (tx == 64 && ty == kPairTY) return f(batch_t<ST, NC, CNS, 64, kPairTY>, batch_occ_t<ST, NC, CNS, 64, kPairTY>);
    } else {
        if (tx == 64 && ty == 8) return f(batch_t<ST, NC, CNS, 64, 8>, batch_occ_t<ST, NC, CNS, 64, 8>);
        if (tx == 32 && ty == 8) return f(batch_t<ST, NC, CNS, 32, 8>, batch_occ_t<ST, NC, CNS, 32, 8>);
    }
    return hipErrorInvalidValue;
}

template <typename F>
static hipError_t batch_dispatch(int storage, int ncomp, int c_ns, int tx, int ty, F&& f)
{
    return by_storage(storage, [&](auto tag) {
        using ST = decltype(tag);
        if (ncomp == 1) return batch_tile<ST, 1, 1>(tx, ty, f);
        if (c_ns == 1) return batch_tile<ST, 2, 1>(tx, ty, f);
        return batch_tile<ST, 2, 2>(tx, ty, f);
    });
}

bool batch_tile_supported(int storage, int ncomp, int tx, int ty)
{
    if (pair_layout(storage, ncomp)) return tx == 64 && ty == kPairTY;
    return (tx == 64 && ty == 8) || (tx == 32 && ty == 8);
}

void batch_default_tile(int storage, int ncomp, int* tx, int* ty)
{
    *tx = 64;
    *ty = pair_layout(storage, ncomp) ? kPairTY : 8;
}

int batch_blocks_per_cu(int storage, int ncomp, int c_ns, int tile_x, int tile_y)
{
    int n = 1;
    (void)batch_dispatch(storage, ncomp, c_ns, tile_x, tile_y, [&](auto, auto occ) {
        n = occ();
        return hipSuccess;
    });
    return n;
}

hipError_t launch_step_batch(int storage, int ncomp, int c_ns, int tile_x, int tile_y, const void* table, int k,
                             int grid, hipStream_t st)
{
    return batch_dispatch(storage, ncomp, c_ns, tile_x, tile_y,
                          [&](auto launch, auto) { return launch(table, k, grid, st); });
}

}  // namespace hm
