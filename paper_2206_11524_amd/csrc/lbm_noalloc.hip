// lbm_totals_get_static: the FP64 totals of lbm_totals_get without any device
// allocation and without the context's scratch, for callers that cannot
// allocate (code under HIP graph capture, tight serving loops).
//
// The per-block partial sums and the totals live in a fixed device array of
// this file, one copy per device, kept until the process ends.  Host code
// never passes the array's name to a kernel: the array's device address is
// looked up once per device with hipGetSymbolAddress and that address is
// passed instead.  Every call on a device shares that device's array, so
// calls that overlap on one device race; each call overwrites every entry it
// reads (nothing needs clearing).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "lbm_internal.h"

namespace {

constexpr int kStaticBlocks = 2048;                       // partial sums of at most this many blocks
constexpr int kStaticDoubles = kStaticBlocks * 5 + 8;     // partials, then the 5 totals
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kStaticDoubles];

std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up once, with
// the device current).
double* scratch_of(int dev)
{
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_ptr[dev] = static_cast<double*>(p);
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" int lbm_totals_get_static(lbm_ctx* c, lbm_totals* tot)
{
    if (!c || !tot) return LBM_EINVAL;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return LBM_EDEVICE;
    if (cur != c->device && hipSetDevice(c->device) != hipSuccess) return LBM_EDEVICE;
    int rc = LBM_OK;
    double* s = scratch_of(c->device);
    double h[5];
    if (!s) {
        rc = LBM_EDEVICE;
    } else if (hm::launch_totals_one_pass(c->prob, c->buf[c->cur], c->ns, s, kStaticBlocks, s + kStaticBlocks * 5,
                                          c->stream) != hipSuccess ||
               hipMemcpyAsync(h, s + kStaticBlocks * 5, sizeof(h), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
               hipStreamSynchronize(c->stream) != hipSuccess) {
        rc = LBM_EDEVICE;
    }
    if (cur != c->device) (void)hipSetDevice(cur);
    if (rc) return rc;
    tot->mass[0] = h[0];
    tot->mass[1] = c->prm.ncomp == 2 ? h[1] : 0.0;
    for (int a = 0; a < 3; ++a) tot->momentum[a] = h[2 + a];
    tot->time = c->t;
    int fin = 1;
    for (double v : h) fin &= std::isfinite(v) ? 1 : 0;
    tot->finite = fin;
    tot->pad = 0;
    return LBM_OK;
}
