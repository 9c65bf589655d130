// Even-odd preconditioned operator and the factor W_eo (C ABI in include/cstar.h).
//
// Paper, mass-reweighting section: D_hat = D_ee - D_eo D_oo^{-1} D_oe on the
// even sites (Q_hat = g5 D_hat), and W_eo = |det[D_oo(m') D_oo(m)^{-1}]|^{1/2},
// computed exactly.  The handle keeps the inverse blocks of (4+m) + SW on the
// odd sites for the last two masses used, and the odd-site scratch vectors.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "cstar_internal.h"

namespace cstar {
namespace {
// Inverse blocks of (4+m) + SW on the odd sites for the two masses used last
// (the mass-reweighting factor alternates between m and m').
struct InvSlot {
    double m = NAN;
    double2 *inv64 = nullptr;
    float4 *inv32 = nullptr;
    long stamp = 0;
};
struct EoState {
    InvSlot slot[2];
    long clock = 0;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    double *partial = nullptr;
};

EoState *state(cstar_gauge *g) {
    if (!g->eo) g->eo = new (std::nothrow) EoState();
    return (EoState *)g->eo;
}

cstar_status ensure_inverse(cstar_gauge *g, EoState *e, double m, InvSlot **out) {
    const long Vh = g->geo.Vh;
    InvSlot *s = nullptr;
    for (InvSlot &c : e->slot)
        if (c.m == m) s = &c;
    if (!s) {
        s = e->slot[0].stamp <= e->slot[1].stamp ? &e->slot[0] : &e->slot[1];
        if (!s->inv64) {
            if (hipMalloc(&s->inv64, sizeof(double2) * 36 * Vh) != hipSuccess ||
                hipMalloc(&s->inv32, sizeof(float4) * 18 * Vh) != hipSuccess) {
                (void)hipGetLastError();
                return fail(CSTAR_ENOMEM, "even-odd: device allocation failed");
            }
        }
        CSTAR_HIP(launch_local_inv(g->geo, g->d, m, s->inv64, s->inv32, g->stream));
        s->m = m;
    }
    s->stamp = ++e->clock;
    *out = s;
    return CSTAR_OK;
}
}  // namespace

void eo_release(cstar_gauge *g) {
    EoState *e = (EoState *)g->eo;
    if (!e) return;
    for (InvSlot &c : e->slot) {
        if (c.inv64) (void)hipFree(c.inv64);
        if (c.inv32) (void)hipFree(c.inv32);
    }
    if (e->tmp) (void)hipFree(e->tmp);
    if (e->partial) (void)hipFree(e->partial);
    delete e;
    g->eo = nullptr;
}

// D_hat(m0) (Q_hat with gamma5) on nrhs even vectors, as dirac_eo_apply (no argument checks).
cstar_status eo_apply(cstar_gauge *g, int nrhs, double m0, cstar_prec prec, int gamma5, const void *in, void *out) {
    const size_t half = cstar_spinor_bytes(g, prec) / 2;
    EoState *e = state(g);
    if (!e) return fail(CSTAR_ENOMEM, "dirac_eo_apply: host allocation failed");
    InvSlot *sl = nullptr;
    cstar_status st = ensure_inverse(g, e, m0, &sl);
    if (st) return st;
    const size_t need = 2 * half * nrhs;
    if (e->tmp_bytes < need) {
        CSTAR_HIP(hipStreamSynchronize(g->stream));
        if (e->tmp) (void)hipFree(e->tmp);
        e->tmp = nullptr;
        e->tmp_bytes = 0;
        if (hipMalloc(&e->tmp, need) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CSTAR_ENOMEM, "dirac_eo_apply: device allocation failed");
        }
        e->tmp_bytes = need;
    }
    EoArgs a{in, e->tmp, out, (long)half, (long)(2 * half), (long)half, nrhs, m0, gamma5 ? 1 : 0,
             prec == CSTAR_FP64 ? (const void *)sl->inv64 : (const void *)sl->inv32};
    CSTAR_HIP(launch_eo_apply(g->geo, g->d, prec, a, g->stream));
    return CSTAR_OK;
}

}  // namespace cstar

using namespace cstar;

extern "C" {

size_t cstar_even_bytes(const cstar_gauge *g, cstar_prec prec) { return cstar_spinor_bytes(g, prec) / 2; }

cstar_status dirac_eo_apply(cstar_gauge *g, int nrhs, double m0, cstar_prec prec, int gamma5, const void *in,
                            void *out) {
    if (!g || !in || !out || nrhs < 1 || !std::isfinite(m0)) return fail(CSTAR_EINVAL, "dirac_eo_apply: bad argument");
    if (prec != CSTAR_FP64 && prec != CSTAR_FP32 && prec != CSTAR_FP32_BF16LINKS)
        return fail(CSTAR_EINVAL, "dirac_eo_apply: bad precision");
    const size_t half = cstar_spinor_bytes(g, prec) / 2;
    const char *ib = (const char *)in, *ob = (const char *)out;
    if (ib < ob + half * nrhs && ob < ib + half * nrhs) return fail(CSTAR_EINVAL, "dirac_eo_apply: in and out overlap");
    return eo_apply(g, nrhs, m0, prec, gamma5, in, out);
}

cstar_status cstar_log_w_eo(cstar_gauge *g, double m, double m_prime, double *log_w_eo) {
    if (!g || !log_w_eo || !std::isfinite(m) || !std::isfinite(m_prime))
        return fail(CSTAR_EINVAL, "cstar_log_w_eo: bad argument");
    EoState *e = state(g);
    if (!e) return fail(CSTAR_ENOMEM, "cstar_log_w_eo: host allocation failed");
    const int nb = eo_pairs_blocks(g->geo);
    if (!e->partial && hipMalloc(&e->partial, sizeof(double) * nb) != hipSuccess) {
        (void)hipGetLastError();
        return fail(CSTAR_ENOMEM, "cstar_log_w_eo: device allocation failed");
    }
    CSTAR_HIP(launch_logdet_ratio(g->geo, g->d, m, m_prime, e->partial, g->stream));
    std::vector<double> hp(nb);
    CSTAR_HIP(hipMemcpyAsync(hp.data(), e->partial, sizeof(double) * nb, hipMemcpyDeviceToHost, g->stream));
    CSTAR_HIP(hipStreamSynchronize(g->stream));
    double sum = 0.0;
    for (double v : hp) sum += v;
    *log_w_eo = sum;
    return CSTAR_OK;
}

}  // extern "C"
