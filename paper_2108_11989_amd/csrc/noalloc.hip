// dirac_apply_noalloc: dirac_apply for callers that cannot allocate device
// memory (declared in include/cstar.h).
//
// dirac_apply stages the per-RHS masses in a device buffer owned by the
// handle.  This variant stages them in `scratch`, a file-scope device array
// of CSTAR_NOALLOC_MAX_RHS doubles that every GPU the library runs on holds
// until the process ends.  Its device address is looked up once per device,
// with that device current, and only that address is handed to copies and
// kernels.  Every call on one GPU shares the array: calls that overlap on one
// GPU (two streams, two threads) race on it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>

#include "cstar_internal.h"

namespace cstar {
namespace {

static __device__ __align__(256) double scratch[CSTAR_NOALLOC_MAX_RHS];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
cstar_status scratch_ptr(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(CSTAR_EDEVICE, "dirac_apply_noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(CSTAR_EDEVICE, std::string("dirac_apply_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
        g_ptr[dev] = (double *)p;
    }
    *out = g_ptr[dev];
    return CSTAR_OK;
}

}  // namespace
}  // namespace cstar

using namespace cstar;

extern "C" cstar_status dirac_apply_noalloc(cstar_gauge *g, int nrhs, const double *masses, cstar_prec prec,
                                            int gamma5, const void *in, void *out) {
    if (!g || !masses || !in || !out || nrhs < 1) return fail(CSTAR_EINVAL, "dirac_apply_noalloc: bad argument");
    if (prec != CSTAR_FP64 && prec != CSTAR_FP32 && prec != CSTAR_FP32_BF16LINKS)
        return fail(CSTAR_EINVAL, "dirac_apply_noalloc: bad precision");
    if (nrhs > CSTAR_NOALLOC_MAX_RHS)
        return fail(CSTAR_EINVAL, "dirac_apply_noalloc: nrhs exceeds CSTAR_NOALLOC_MAX_RHS (" +
                                      std::to_string(CSTAR_NOALLOC_MAX_RHS) + ")");
    for (int j = 0; j < nrhs; j++)
        if (!std::isfinite(masses[j])) return fail(CSTAR_EINVAL, "dirac_apply_noalloc: non-finite mass");
    const size_t bytes = cstar_spinor_bytes(g, prec);
    const char *ib = (const char *)in, *ob = (const char *)out;
    if (ib < ob + bytes * nrhs && ob < ib + bytes * nrhs)
        return fail(CSTAR_EINVAL, "dirac_apply_noalloc: in and out overlap");
    int cur = -1;
    CSTAR_HIP(hipGetDevice(&cur));
    if (cur != g->device) CSTAR_HIP(hipSetDevice(g->device));
    double *m_dev = nullptr;
    cstar_status st = scratch_ptr(g->device, &m_dev);
    if (st == CSTAR_OK) {
        ApplyArgs a{in, out, (long)bytes, nrhs, gamma5 ? 1 : 0, m_dev, masses[0]};
        a.no_tune = 1;
        hipError_t e = hipMemcpyAsync(m_dev, masses, sizeof(double) * nrhs, hipMemcpyHostToDevice, g->stream);
        if (e == hipSuccess) e = handle_apply(g, prec, a);
        if (e != hipSuccess) st = fail(CSTAR_EDEVICE, std::string("dirac_apply_noalloc: ") + hipGetErrorString(e));
    }
    if (cur != g->device) (void)hipSetDevice(cur);
    return st;
}
