// Host runtime of the HMCSC library: the C ABI of include/lbm.h on top of the
// HIP kernels.  One context = one periodic D3Q19 domain on one device, its two
// population buffers (A -> B, swapped every step), the n_s field, and a scratch
// area for FP64 diagnostics and checkpoint staging.
#include "lbm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "lbm_internal.h"

namespace hm_rt {

int validate(const lbm_domain* d, const lbm_params* p)
{
    if (!d || !p) return LBM_EINVAL;
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return LBM_EINVAL;
    // each plane block of 19 direction arrays is addressed through one
    // buffer descriptor with 32-bit offsets
    const int64_t plane = static_cast<int64_t>(d->nx) * d->ny;
    if (plane * hm::kQ * 8 >= (int64_t(1) << 32)) return LBM_EINVAL;
    if (static_cast<int64_t>(d->nz) * plane >= (int64_t(1) << 40)) return LBM_EINVAL;
    if (p->ncomp < 1 || p->ncomp > 2) return LBM_EINVAL;
    if (p->c_ns < 1 || p->c_ns > 2 || p->c_ns > p->ncomp) return LBM_EINVAL;
    for (int s = 0; s < p->ncomp; ++s) {
        if (!(p->tau[s] > 0.5) || !std::isfinite(p->tau[s])) return LBM_EINVAL;
        if (!std::isfinite(p->G_ads[s]) || !std::isfinite(p->rho_shift[s])) return LBM_EINVAL;
    }
    if (!std::isfinite(p->G_inter) || !std::isfinite(p->g_scale)) return LBM_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p->F_ext[a])) return LBM_EINVAL;
    if (p->storage < LBM_F64 || p->storage > LBM_BF16S) return LBM_EINVAL;
    if (p->store_scale_log2 < -30 || p->store_scale_log2 > 30) return LBM_EINVAL;
    if ((p->storage == LBM_F64 || p->storage == LBM_F32) && p->store_scale_log2 != 0) return LBM_EINVAL;
    if (p->n_res < 0 || p->n_res > LBM_MAX_RES) return LBM_EINVAL;
    const int dims[3] = {d->nx, d->ny, d->nz};
    for (int r = 0; r < p->n_res; ++r) {
        const lbm_reservoir& R = p->res[r];
        if (R.axis < 0 || R.axis > 2 || R.lo < 0 || R.hi < R.lo || R.hi > dims[R.axis]) return LBM_EINVAL;
        for (int s = 0; s < p->ncomp; ++s)
            if (!std::isfinite(R.rho[s])) return LBM_EINVAL;
    }
    if (p->check_every < 0) return LBM_EINVAL;
    if (p->rounding != LBM_ROUND_NEAREST && p->rounding != LBM_ROUND_STOCHASTIC) return LBM_EINVAL;
    if (p->forcing != LBM_FORCING_SHAN_CHEN && p->forcing != LBM_FORCING_GUO) return LBM_EINVAL;
    return LBM_OK;
}

hm::Problem make_problem(const lbm_domain* d, const lbm_params* p)
{
    hm::Problem q{};
    q.nx = d->nx; q.ny = d->ny; q.nz = d->nz;
    q.N = static_cast<int64_t>(d->nx) * d->ny * d->nz;
    q.ncomp = p->ncomp; q.c_ns = p->c_ns; q.storage = p->storage;
    for (int s = 0; s < 2; ++s) {
        q.tau[s] = s < p->ncomp ? p->tau[s] : 1.0;
        q.Gads_s[s] = s < p->ncomp ? p->G_ads[s] * p->g_scale : 0.0;
        q.rho0[s] = s < p->ncomp ? p->rho_shift[s] : 0.0;
    }
    q.G_s = p->G_inter * p->g_scale;
    q.g_scale = p->g_scale;
    q.G_inter = p->G_inter;
    for (int a = 0; a < 3; ++a) q.F[a] = p->F_ext[a];
    q.scale = std::ldexp(1.0, p->store_scale_log2);
    q.stochastic = (p->storage == LBM_F16S || p->storage == LBM_BF16S) && p->rounding == LBM_ROUND_STOCHASTIC;
    q.forcing = p->forcing == LBM_FORCING_GUO ? hm::kForcingGuo : hm::kForcingShanChen;
    q.n_res = p->n_res;
    for (int r = 0; r < hm::kMaxRes; ++r) {
        if (r < p->n_res) {
            q.res_axis[r] = p->res[r].axis; q.res_lo[r] = p->res[r].lo; q.res_hi[r] = p->res[r].hi;
            q.res_rho[r][0] = p->res[r].rho[0];
            q.res_rho[r][1] = p->ncomp == 2 ? p->res[r].rho[1] : 0.0;
        } else {
            q.res_axis[r] = 0; q.res_lo[r] = 0; q.res_hi[r] = 0;
            q.res_rho[r][0] = q.res_rho[r][1] = 0.0;
        }
    }
    return q;
}

int env_int(const char* name, int dflt)
{
    const char* v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v);
}

hm::Launch choose_launch(const hm::Problem& p, int cus)
{
    hm::Launch l{};
    // FP64 with two components needs the smaller tile to stay within the
    // register file (no spills); the pair kernel runs one thread per cell
    // plus three ring waves on 64-wide tiles of pair_tile_y() rows
    const bool wide = p.storage == hm::kF64 && p.ncomp == 2;
    const bool pair = hm::pair_layout(p.storage, p.ncomp, p.forcing);
    const int pty = hm::pair_tile_y();
    const int dflt_y = pair ? (p.ny >= pty ? pty : 4) : ((p.ny >= 8 && !wide) ? 8 : 4);
    l.tile_x = env_int("LBM_TILE_X", 64);
    l.tile_y = env_int("LBM_TILE_Y", dflt_y);
    // the GS-WBS and one-plane domains use the default tile widths only
    if (!hm::tile_supported(p.storage, p.ncomp, l.tile_x, l.tile_y, p.forcing) ||
        ((p.forcing == hm::kForcingGuo || p.nz == 1) &&
         !(l.tile_x == 64 && (pair ? (l.tile_y == pty || l.tile_y == 4) : (l.tile_y == 8 || l.tile_y == 4))))) {
        l.tile_x = 64;
        l.tile_y = dflt_y;
    }
    const int ntx = (p.nx + l.tile_x - 1) / l.tile_x;
    const int nty = (p.ny + l.tile_y - 1) / l.tile_y;
    const int64_t cols = static_cast<int64_t>(ntx) * nty;
    int zc = env_int("LBM_ZCHUNK", 0);
    if (zc <= 0) {
        // One block fits a CU (registers and LDS), so blocks run in rounds
        // of one per CU, and a block takes about (chunk + 8) plane times: the
        // halo planes, the pipeline fill and drain and the block's start cost
        // as much as about eight planes (fitted to timings of 192^3 to 384^3
        // domains).  Take the chunking with the least rounds x (chunk + 8),
        // the fewest chunks among equals.
        // Chunks shorter than 16 planes spend too much on their halo, unless
        // the domain would then give fewer than two such tiles per CU: a
        // small domain would leave most CUs idle, and its halo re-reads are
        // L2 hits.
        const int64_t ncu = std::max(cus, 1);
        const int64_t tiles16 = cols * ((p.nz + 15) / 16);
        const int64_t min_chunk = tiles16 >= 2 * ncu ? 16 : 4;
        int64_t best_cost = -1;
        for (int64_t c = 1; c <= p.nz; ++c) {
            const int64_t z = (p.nz + c - 1) / c;
            if (c > 1 && z < min_chunk) break;
            const int64_t blocks = cols * ((p.nz + z - 1) / z);
            const int64_t cost = ((blocks + ncu - 1) / ncu) * (z + 8);
            if (best_cost < 0 || cost < best_cost) {
                best_cost = cost;
                zc = static_cast<int>(z);
            }
        }
    }
    l.zchunk = std::min(std::max(zc, 1), p.nz);
    return l;
}

}  // namespace hm_rt

using namespace hm_rt;

#define HIP_TRY(expr)                                  \
    do {                                               \
        if ((expr) != hipSuccess) return LBM_EDEVICE;  \
    } while (0)

int hm_rt::compute_totals(lbm_ctx* c, bool fields, bool forces, lbm_totals* tot)
{
    double* rho = reinterpret_cast<double*>(c->scratch + c->sl.rho);
    double* u = reinterpret_cast<double*>(c->scratch + c->sl.u);
    double* p = reinterpret_cast<double*>(c->scratch + c->sl.p);
    double* part = reinterpret_cast<double*>(c->scratch + c->sl.partials);
    double* tots = reinterpret_cast<double*>(c->scratch + c->sl.totals);
    HIP_TRY(hm::launch_diagnostics(c->prob, c->buf[c->cur], c->ns, forces || fields, rho, fields ? u : nullptr,
                                   fields ? p : nullptr, part, tots, c->stream));
    double h[5];
    HIP_TRY(hipMemcpyAsync(h, tots, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (tot) {
        tot->mass[0] = h[0];
        tot->mass[1] = c->prm.ncomp == 2 ? h[1] : 0.0;
        for (int a = 0; a < 3; ++a) tot->momentum[a] = h[2 + a];
        tot->time = c->t;
        int fin = 1;
        for (double v : h) fin &= std::isfinite(v) ? 1 : 0;
        tot->finite = fin;
        tot->pad = 0;
    }
    return LBM_OK;
}

extern "C" {

const char* lbm_strerror(int code)
{
    switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of memory";
    case LBM_EDEVICE: return "HIP device error";
    case LBM_EUNSTABLE: return "non-finite state (unstable simulation)";
    case LBM_ENOTFOUND: return "unknown ticket";
    case LBM_EAGAIN: return "not ready";
    default: return "unknown error";
    }
}

int lbm_required_bytes(const lbm_domain* d, const lbm_params* p, lbm_sizes* out)
{
    const int rc = validate(d, p);
    if (rc) return rc;
    if (!out) return LBM_EINVAL;
    const int64_t N = static_cast<int64_t>(d->nx) * d->ny * d->nz;
    out->pop_bytes = align_up(static_cast<size_t>(hm::storage_bytes(p->storage)) * hm::kQ * p->ncomp * N);
    out->ns_bytes = align_up(sizeof(float) * static_cast<size_t>(p->c_ns) * N);
    out->scratch_bytes = scratch_layout(N, p->ncomp).bytes;
    return LBM_OK;
}

static void free_owned(lbm_ctx* c)
{
    if (!c->owned) return;
    if (c->buf[0]) (void)hipFree(c->buf[0]);
    if (c->buf[1]) (void)hipFree(c->buf[1]);
    if (c->ns) (void)hipFree(c->ns);
    if (c->scratch) (void)hipFree(c->scratch);
    c->buf[0] = c->buf[1] = nullptr;
    c->ns = nullptr;
    c->scratch = nullptr;
}

void lbm_destroy(lbm_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_owned(c);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    delete c;
}

int lbm_create(const lbm_domain* dom, const float* n_s, const double* rho_init, const lbm_params* prm,
               const lbm_device_buffers* bufs, void* stream, lbm_ctx** out)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    int rc = validate(dom, prm);
    if (rc) return rc;
    if (!n_s || !rho_init) return LBM_EINVAL;
    const int64_t N = static_cast<int64_t>(dom->nx) * dom->ny * dom->nz;
    for (int64_t k = 0; k < static_cast<int64_t>(prm->c_ns) * N; ++k)
        if (!(n_s[k] >= 0.0f && n_s[k] <= 1.0f)) return LBM_EINVAL;
    for (int64_t k = 0; k < static_cast<int64_t>(prm->ncomp) * N; ++k)
        if (!std::isfinite(rho_init[k])) return LBM_EINVAL;
    if (bufs && (!bufs->f_a || !bufs->f_b || !bufs->n_s || !bufs->scratch)) return LBM_EINVAL;
    if (bufs) {
        const void* ps[4] = {bufs->f_a, bufs->f_b, bufs->n_s, bufs->scratch};
        for (const void* q : ps)
            if (reinterpret_cast<uintptr_t>(q) % kAlign) return LBM_EINVAL;
    }

    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return LBM_ENOMEM;
    c->dom = *dom;
    c->prm = *prm;
    c->prob = make_problem(dom, prm);

    lbm_required_bytes(dom, prm, &c->sizes);
    c->sl = scratch_layout(N, prm->ncomp);
    c->stream = static_cast<hipStream_t>(stream);
    c->cur = 0;
    c->t = 0;
    if (hipGetDevice(&c->device) != hipSuccess) { delete c; return LBM_EDEVICE; }
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
        delete c;
        return LBM_EDEVICE;
    }
    c->launch = choose_launch(c->prob, cus);
    if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        lbm_destroy(c);
        return LBM_EDEVICE;
    }
    if (bufs) {
        c->owned = false;
        c->buf[0] = bufs->f_a;
        c->buf[1] = bufs->f_b;
        c->ns = static_cast<float*>(bufs->n_s);
        c->scratch = static_cast<char*>(bufs->scratch);
    } else {
        c->owned = true;
        if (hipMalloc(&c->buf[0], c->sizes.pop_bytes) != hipSuccess ||
            hipMalloc(&c->buf[1], c->sizes.pop_bytes) != hipSuccess ||
            hipMalloc(reinterpret_cast<void**>(&c->ns), c->sizes.ns_bytes) != hipSuccess ||
            hipMalloc(reinterpret_cast<void**>(&c->scratch), c->sizes.scratch_bytes) != hipSuccess) {
            (void)hipGetLastError();
            lbm_destroy(c);
            return LBM_ENOMEM;
        }
    }
    // n_s and the initial densities; the densities are staged in the rho slot of scratch
    double* rho_dev = reinterpret_cast<double*>(c->scratch + c->sl.rho);
    if (hipMemcpyAsync(c->ns, n_s, sizeof(float) * prm->c_ns * N, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
        hipMemcpyAsync(rho_dev, rho_init, sizeof(double) * prm->ncomp * N, hipMemcpyHostToDevice, c->stream) !=
            hipSuccess ||
        hm::launch_init(c->prob, rho_dev, c->buf[0], c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess) {
        lbm_destroy(c);
        return LBM_EDEVICE;
    }
    *out = c;
    return LBM_OK;
}

}  // extern "C"

// A context over caller buffers that already hold (or will receive) its
// state: no device work, no synchronisation (the server initialises the
// state itself, on its admission stream).
int hm_rt::ctx_bind(const lbm_domain* dom, const lbm_params* prm, const lbm_device_buffers* bufs, hipStream_t stream,
                    lbm_ctx** out)
{
    *out = nullptr;
    int rc = validate(dom, prm);
    if (rc) return rc;
    if (!bufs || !bufs->f_a || !bufs->f_b || !bufs->n_s || !bufs->scratch) return LBM_EINVAL;
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return LBM_ENOMEM;
    c->dom = *dom;
    c->prm = *prm;
    c->prob = make_problem(dom, prm);
    lbm_required_bytes(dom, prm, &c->sizes);
    c->sl = scratch_layout(c->prob.N, prm->ncomp);
    c->stream = stream;
    c->cur = 0;
    c->t = 0;
    c->owned = false;
    c->buf[0] = bufs->f_a;
    c->buf[1] = bufs->f_b;
    c->ns = static_cast<float*>(bufs->n_s);
    c->scratch = static_cast<char*>(bufs->scratch);
    int cus = 0;
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        lbm_destroy(c);
        return LBM_EDEVICE;
    }
    c->launch = choose_launch(c->prob, cus);
    *out = c;
    return LBM_OK;
}

extern "C" {

int lbm_step(lbm_ctx* c, int64_t nsteps)
{
    if (!c || nsteps < 0) return LBM_EINVAL;
    if (nsteps == 0) return LBM_OK;
    HIP_TRY(hipEventRecord(c->ev0, c->stream));
    for (int64_t k = 0; k < nsteps; ++k) {
        HIP_TRY(hm::launch_step(c->prob, c->launch, c->t, c->buf[c->cur], c->buf[1 - c->cur], c->ns, c->stream));
        c->cur = 1 - c->cur;
        c->t += 1;
        if (c->prm.check_every > 0 && c->t % c->prm.check_every == 0) {
            lbm_totals tt;
            const int rc = compute_totals(c, false, false, &tt);
            if (rc) return rc;
            if (!tt.finite) return LBM_EUNSTABLE;
        }
    }
    HIP_TRY(hipEventRecord(c->ev1, c->stream));
    c->timed_steps = nsteps;
    return LBM_OK;
}

double lbm_last_step_ms(const lbm_ctx* c)
{
    if (!c || c->timed_steps <= 0) return 0.0;
    if (hipEventSynchronize(c->ev1) != hipSuccess) return 0.0;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, c->ev0, c->ev1) != hipSuccess) return 0.0;
    return static_cast<double>(ms) / static_cast<double>(c->timed_steps);
}

int lbm_moments(lbm_ctx* c, double* rho, double* u, double* p, lbm_totals* tot)
{
    if (!c) return LBM_EINVAL;
    const bool fields = rho || u || p;
    const int rc = compute_totals(c, fields, true, tot);
    if (rc) return rc;
    const int64_t N = c->prob.N;
    if (rho)
        HIP_TRY(hipMemcpy(rho, c->scratch + c->sl.rho, sizeof(double) * c->prm.ncomp * N, hipMemcpyDeviceToHost));
    if (u) HIP_TRY(hipMemcpy(u, c->scratch + c->sl.u, sizeof(double) * 3 * N, hipMemcpyDeviceToHost));
    if (p) HIP_TRY(hipMemcpy(p, c->scratch + c->sl.p, sizeof(double) * N, hipMemcpyDeviceToHost));
    return LBM_OK;
}

int lbm_totals_get(lbm_ctx* c, lbm_totals* tot)
{
    if (!c || !tot) return LBM_EINVAL;
    return compute_totals(c, false, true, tot);
}

int lbm_get_populations(lbm_ctx* c, double* f)
{
    if (!c || !f) return LBM_EINVAL;
    const int64_t N = c->prob.N;
    double* stage = reinterpret_cast<double*>(c->scratch + c->sl.u);  // N doubles (u slot holds 3N)
    for (int s = 0; s < c->prm.ncomp; ++s)
        for (int i = 0; i < hm::kQ; ++i) {
            HIP_TRY(hm::launch_canonical(c->prob, c->buf[c->cur], s, i, stage, c->stream));
            HIP_TRY(hipMemcpyAsync(f + static_cast<size_t>(s * hm::kQ + i) * N, stage, sizeof(double) * N,
                                   hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
        }
    return LBM_OK;
}

int lbm_set_populations(lbm_ctx* c, const double* f)
{
    if (!c || !f) return LBM_EINVAL;
    const int64_t N = c->prob.N;
    for (int64_t k = 0; k < static_cast<int64_t>(c->prm.ncomp) * hm::kQ * N; ++k)
        if (!std::isfinite(f[k])) return LBM_EINVAL;
    double* stage = reinterpret_cast<double*>(c->scratch + c->sl.u);
    for (int s = 0; s < c->prm.ncomp; ++s)
        for (int i = 0; i < hm::kQ; ++i) {
            HIP_TRY(hipMemcpyAsync(stage, f + static_cast<size_t>(s * hm::kQ + i) * N, sizeof(double) * N,
                                   hipMemcpyHostToDevice, c->stream));
            HIP_TRY(hm::launch_set_canonical(c->prob, stage, s, i, c->buf[c->cur], c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
        }
    return LBM_OK;
}

int lbm_set_reservoir(lbm_ctx* c, int32_t r, const double rho[2])
{
    if (!c || !rho || r < 0 || r >= c->prm.n_res) return LBM_EINVAL;
    for (int s = 0; s < c->prm.ncomp; ++s)
        if (!std::isfinite(rho[s])) return LBM_EINVAL;
    for (int s = 0; s < c->prm.ncomp; ++s) {
        c->prm.res[r].rho[s] = rho[s];
        c->prob.res_rho[r][s] = rho[s];
    }
    return LBM_OK;
}

int lbm_fill_state_get(lbm_ctx* c, const lbm_fill_query* q, lbm_fill_state* out)
{
    if (!c || !q || !out) return LBM_EINVAL;
    if (q->axis < 0 || q->axis > 2 || q->comp < 0 || q->comp >= c->prm.ncomp) return LBM_EINVAL;
    const int len = q->axis == 0 ? c->dom.nx : (q->axis == 1 ? c->dom.ny : c->dom.nz);
    auto slab_ok = [&](int lo, int hi, bool nonempty) { return lo >= 0 && hi <= len && (nonempty ? lo < hi : lo <= hi); };
    if (!slab_ok(q->inlet_lo, q->inlet_hi, true) || !slab_ok(q->outlet_lo, q->outlet_hi, true) ||
        !slab_ok(q->pore_lo, q->pore_hi, false) || !std::isfinite(q->threshold))
        return LBM_EINVAL;
    const int rc = compute_totals(c, true, true, nullptr);  // FP64 densities and pressure into the scratch
    if (rc) return rc;
    hm::FillQuery f{q->axis, q->inlet_lo, q->inlet_hi, q->outlet_lo, q->outlet_hi, q->pore_lo, q->pore_hi, q->comp,
                    q->threshold};
    double* part = reinterpret_cast<double*>(c->scratch + c->sl.partials);
    double* tots = reinterpret_cast<double*>(c->scratch + c->sl.totals);
    HIP_TRY(hm::launch_fill(c->prob, f, reinterpret_cast<const double*>(c->scratch + c->sl.rho),
                            reinterpret_cast<const double*>(c->scratch + c->sl.p), c->ns, part, tots, c->stream));
    double h[6];
    HIP_TRY(hipMemcpyAsync(h, tots, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    out->p_inlet = h[0] / h[1];
    out->p_outlet = h[2] / h[3];
    out->dp = out->p_inlet - out->p_outlet;
    out->saturation = h[5] > 0.0 ? h[4] / h[5] : 0.0;
    out->pore_volume = h[5];
    out->time = c->t;
    return LBM_OK;
}

int lbm_permeability_get(lbm_ctx* c, int32_t axis, lbm_permeability* out)
{
    if (!c || !out || axis < 0 || axis > 2) return LBM_EINVAL;
    const double F = c->prm.F_ext[axis];
    if (F == 0.0 || (c->prm.ncomp == 2 && c->prm.tau[0] != c->prm.tau[1])) return LBM_EINVAL;
    const int rc = compute_totals(c, true, true, nullptr);  // FP64 densities and u_macro into the scratch
    if (rc) return rc;
    double* part = reinterpret_cast<double*>(c->scratch + c->sl.partials);
    double* tots = reinterpret_cast<double*>(c->scratch + c->sl.totals);
    HIP_TRY(hm::launch_flux(c->prob, axis, reinterpret_cast<const double*>(c->scratch + c->sl.rho),
                            reinterpret_cast<const double*>(c->scratch + c->sl.u), part, tots, c->stream));
    double h[3];
    HIP_TRY(hipMemcpyAsync(h, tots, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const double N = static_cast<double>(c->prob.N);
    const double nu = (c->prm.tau[0] - 0.5) / 3.0;
    out->nu = nu;
    out->momentum = h[2] / N;
    out->k = nu * out->momentum / F;
    out->k_comp[0] = nu * (h[0] / N) / F;
    out->k_comp[1] = c->prm.ncomp == 2 ? nu * (h[1] / N) / F : 0.0;
    out->time = c->t;
    return LBM_OK;
}

int lbm_droplet_get(lbm_ctx* c, const lbm_droplet_query* q, lbm_droplet_state* out)
{
    if (!c || !q || !out || q->comp < 0 || q->comp >= c->prm.ncomp) return LBM_EINVAL;
    for (double v : q->center)
        if (!std::isfinite(v)) return LBM_EINVAL;
    if (!(q->r_core > 0.0) || !(q->r_far > q->r_core) || !(q->margin >= 0.0) || !std::isfinite(q->r_far) ||
        !std::isfinite(q->margin))
        return LBM_EINVAL;
    lbm_totals tot{};
    const int rc = compute_totals(c, true, true, &tot);  // FP64 densities and pressure into the scratch
    if (rc) return rc;
    const int64_t N = c->prob.N;
    const double* rho = reinterpret_cast<const double*>(c->scratch + c->sl.rho) + static_cast<size_t>(q->comp) * N;
    const double* pr = reinterpret_cast<const double*>(c->scratch + c->sl.p);
    double* part = reinterpret_cast<double*>(c->scratch + c->sl.partials);
    double* tots = reinterpret_cast<double*>(c->scratch + c->sl.totals);
    double h[4];
    auto ball = [&](const double* f, double r_in, double r_out) -> int {
        HIP_TRY(hm::launch_ball(c->prob, q->center, r_in, r_out, f, part, tots, c->stream));
        HIP_TRY(hipMemcpyAsync(h, tots, sizeof(h), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipStreamSynchronize(c->stream));
        return (h[1] > 0.0 && h[3] > 0.0) ? LBM_OK : LBM_EINVAL;
    };
    int r = ball(rho, q->r_core, q->r_far);
    if (r) return r;
    const double rho_in = h[0] / h[1], rho_out = h[2] / h[3];
    if (!(std::fabs(rho_in - rho_out) > 0.0)) return LBM_EINVAL;
    const double V = (tot.mass[q->comp] - rho_out * static_cast<double>(N)) / (rho_in - rho_out);
    if (!(V > 0.0)) return LBM_EINVAL;
    const bool two_d = c->dom.nz == 1;
    const double pi = 3.14159265358979323846;
    const double R = two_d ? std::sqrt(V / pi) : std::cbrt(3.0 * V / (4.0 * pi));
    r = ball(pr, R / 2.0, R + q->margin);
    if (r) return r;
    out->R = R;
    out->rho_in = rho_in;
    out->rho_out = rho_out;
    out->p_in = h[0] / h[1];
    out->p_out = h[2] / h[3];
    out->dp = out->p_in - out->p_out;
    out->gamma = two_d ? out->dp * R : out->dp * R / 2.0;
    out->time = c->t;
    return LBM_OK;
}

int64_t lbm_time(const lbm_ctx* c) { return c ? c->t : -1; }

int lbm_set_time(lbm_ctx* c, int64_t t)
{
    if (!c || t < 0) return LBM_EINVAL;
    c->t = t;
    return LBM_OK;
}

int lbm_sync(lbm_ctx* c)
{
    if (!c) return LBM_EINVAL;
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

}  // extern "C"
