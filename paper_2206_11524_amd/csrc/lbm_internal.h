// Internal declarations shared by the host runtime files of the HMCSC
// library (not part of the public ABI, which is include/lbm.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lbm.h"
#include "lbm_kernels.h"

namespace hm_rt {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Scratch layout: [rho ncomp*N][u 3N][p N][partials][totals 5] (FP64).
struct ScratchLayout {
    size_t rho, u, p, partials, totals, bytes;
};

inline ScratchLayout scratch_layout(int64_t N, int ncomp)
{
    ScratchLayout s{};
    size_t off = 0;
    s.rho = off; off = align_up(off + sizeof(double) * static_cast<size_t>(ncomp) * N);
    s.u = off; off = align_up(off + sizeof(double) * 3 * static_cast<size_t>(N));
    s.p = off; off = align_up(off + sizeof(double) * static_cast<size_t>(N));
    s.partials = off; off = align_up(off + sizeof(double) * 10 * hm::moments_max_blocks());
    s.totals = off; off = align_up(off + sizeof(double) * 6);
    s.bytes = off;
    return s;
}

int validate(const lbm_domain* d, const lbm_params* p);
int env_int(const char* name, int dflt);
hm::Problem make_problem(const lbm_domain* d, const lbm_params* p);
hm::Launch choose_launch(const hm::Problem& p, int cus);

}  // namespace hm_rt

struct lbm_ctx {
    lbm_domain dom;
    lbm_params prm;
    hm::Problem prob;
    hm::Launch launch;
    lbm_sizes sizes;
    hm_rt::ScratchLayout sl;
    void* buf[2];
    float* ns;
    char* scratch;
    bool owned;
    hipStream_t stream;
    int device;
    int cur;  // index of the buffer holding the current state
    int64_t t;
    hipEvent_t ev0, ev1;
    int64_t timed_steps;
};

namespace hm_rt {
// A context over caller buffers, without any device work (see lbm_runtime.cpp).
int ctx_bind(const lbm_domain* dom, const lbm_params* prm, const lbm_device_buffers* bufs, hipStream_t stream,
             lbm_ctx** out);

// FP64 totals (and, if fields, per-cell moments into scratch) of the current
// state.  With forces false only the mass and the local part of the momentum
// are summed (the health check).
int compute_totals(lbm_ctx* c, bool fields, bool forces, lbm_totals* tot);
}  // namespace hm_rt
