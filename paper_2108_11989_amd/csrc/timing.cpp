// Event timing of the Dirac-apply launches of one handle (cstar_timing_* in cstar.h).
#include <hip/hip_runtime.h>

#include <vector>

#include "cstar_internal.h"

namespace cstar {

namespace {
struct Pending {
    hipEvent_t a, b;
    int prec;
};
struct Timing {
    long launches[3] = {0, 0, 0};
    long rhs[3] = {0, 0, 0};
    long operands[3] = {0, 0, 0};
    double ms[3] = {0, 0, 0};
    std::vector<Pending> pending;
    std::vector<hipEvent_t> pool;
};

hipEvent_t take(Timing *t) {
    if (!t->pool.empty()) {
        hipEvent_t e = t->pool.back();
        t->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

hipError_t drain(Timing *t) {
    for (const Pending &p : t->pending) {
        hipError_t e = hipEventSynchronize(p.b);
        if (e != hipSuccess) return e;
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e != hipSuccess) return e;
        t->ms[p.prec] += ms;
        t->pool.push_back(p.a);
        t->pool.push_back(p.b);
    }
    t->pending.clear();
    return hipSuccess;
}
}  // namespace

hipError_t handle_apply(cstar_gauge *g, cstar_prec prec, const ApplyArgs &a) {
    Timing *t = (Timing *)g->timing;
    if (!t) return launch_apply(g->geo, g->d, prec, a, g->stream);
    hipEvent_t ea = take(t), eb = take(t);
    if (!ea || !eb) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(ea, g->stream);
    if (e == hipSuccess) e = launch_apply(g->geo, g->d, prec, a, g->stream);
    if (e == hipSuccess) e = hipEventRecord(eb, g->stream);
    if (e != hipSuccess) return e;
    t->pending.push_back({ea, eb, (int)prec});
    t->launches[prec] += 1;
    t->rhs[prec] += a.nrhs;
    t->operands[prec] += (long)a.nrhs * ((a.y ? 1 : 0) + (a.z ? 1 : 0) + (a.w ? 1 : 0));
    if (t->pending.size() >= 4096) return drain(t);
    return hipSuccess;
}

void timing_release(cstar_gauge *g) {
    Timing *t = (Timing *)g->timing;
    if (!t) return;
    (void)drain(t);
    for (hipEvent_t e : t->pool) (void)hipEventDestroy(e);
    delete t;
    g->timing = nullptr;
}

}  // namespace cstar

using namespace cstar;

extern "C" cstar_status cstar_timing_enable(cstar_gauge *g, int on) {
    if (!g) return fail(CSTAR_EINVAL, "cstar_timing_enable: null handle");
    timing_release(g);
    if (on) g->timing = new Timing();
    return CSTAR_OK;
}

extern "C" cstar_status cstar_timing_read(cstar_gauge *g, cstar_apply_timing *out) {
    if (!g || !out) return fail(CSTAR_EINVAL, "cstar_timing_read: bad argument");
    Timing *t = (Timing *)g->timing;
    *out = cstar_apply_timing{};
    if (!t) return CSTAR_OK;
    CSTAR_HIP(drain(t));
    for (int p = 0; p < 3; p++) {
        out->launches[p] = t->launches[p];
        out->rhs[p] = t->rhs[p];
        out->ms[p] = t->ms[p];
        out->operands[p] = t->operands[p];
    }
    return CSTAR_OK;
}
