// C ABI of libcstar (declarations and argument contracts in include/cstar.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cstar_internal.h"
#include "eig.h"

namespace cstar {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }
cstar_status fail(cstar_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

cstar_status sign_driver(cstar_eig_provider prov, void *ctx, const double *m_path, int n, int k, double c,
                         double m_max, int *sign_out, cstar_sign_report *report);

static void free_gauge_dev(GaugeDev &d) {
    void *ptrs[] = {d.link64, d.link32, d.linkbf_a, d.linkbf_b, d.phase32, d.clov64, d.clov32};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    d = GaugeDev();
}

}  // namespace cstar

using namespace cstar;

namespace {
struct MassBuf {
    double *dev = nullptr;
    int cap = 0;
};
// per-handle mass staging buffer, kept beside the handle
struct HandleExtra {
    MassBuf masses;
};
}  // namespace

extern "C" {

const char *cstar_last_error(void) { return g_err.c_str(); }

cstar_status cstar_gauge_create(const cstar_params *par, const double *su3, const double *theta, int src_on_device,
                                void *stream, cstar_gauge **out) {
    if (!par || !su3 || !theta || !out) return fail(CSTAR_EINVAL, "cstar_gauge_create: null argument");
    *out = nullptr;
    if (par->T < 2 || par->L < 2 || (par->T & 1) || (par->L & 1))
        return fail(CSTAR_EINVAL, "cstar_gauge_create: T and L must be even and >= 2");
    if (par->time_bc != 1 && par->time_bc != -1) return fail(CSTAR_EINVAL, "cstar_gauge_create: time_bc must be +-1");
    if (!std::isfinite(par->q) || !std::isfinite(par->csw_su3) || !std::isfinite(par->csw_u1))
        return fail(CSTAR_EINVAL, "cstar_gauge_create: non-finite parameter");
    const long V = (long)par->T * par->L * par->L * par->L;
    if (V / 2 > (1L << 28)) return fail(CSTAR_EINVAL, "cstar_gauge_create: lattice too large");
    const size_t n_su3 = (size_t)V * 4 * 18, n_th = (size_t)V * 4;
    if (!src_on_device) {
        for (size_t i = 0; i < n_su3; i++)
            if (!std::isfinite(su3[i])) return fail(CSTAR_EINVAL, "cstar_gauge_create: non-finite link entry");
        for (size_t i = 0; i < n_th; i++)
            if (!std::isfinite(theta[i])) return fail(CSTAR_EINVAL, "cstar_gauge_create: non-finite U(1) angle");
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(CSTAR_EDEVICE, "no HIP device");
    cstar_gauge *g = new (std::nothrow) cstar_gauge();
    if (!g) return fail(CSTAR_ENOMEM, "host allocation failed");
    g->par = *par;
    g->geo.T = par->T;
    g->geo.L = par->L;
    g->geo.Lh = par->L / 2;
    g->geo.Vh = (int)(V / 2);
    g->geo.time_bc = par->time_bc;
    (void)hipGetDevice(&g->device);
    g->stream = (hipStream_t)stream;
    const long Vh = g->geo.Vh;
    GaugeDev &d = g->d;
    double *su3_d = nullptr, *th_d = nullptr, *partial = nullptr;
    bool ok = hipMalloc(&d.link64, sizeof(double2) * 2 * 4 * 9 * Vh) == hipSuccess &&
              hipMalloc(&d.link32, sizeof(float4) * 2 * 4 * 3 * Vh) == hipSuccess &&
              hipMalloc(&d.linkbf_a, sizeof(uint4) * 2 * 4 * Vh) == hipSuccess &&
              hipMalloc(&d.linkbf_b, sizeof(uint2) * 2 * 4 * Vh) == hipSuccess &&
              hipMalloc(&d.phase32, sizeof(float2) * 2 * 4 * Vh) == hipSuccess &&
              hipMalloc(&d.clov64, sizeof(double2) * 2 * 36 * Vh) == hipSuccess &&
              hipMalloc(&d.clov32, sizeof(float4) * 2 * 18 * Vh) == hipSuccess &&
              hipMalloc(&partial, sizeof(double) * clover_norm_blocks(g->geo)) == hipSuccess;
    if (ok && !src_on_device)
        ok = hipMalloc(&su3_d, sizeof(double) * n_su3) == hipSuccess &&
             hipMalloc(&th_d, sizeof(double) * n_th) == hipSuccess;
    auto cleanup = [&]() {
        (void)hipGetLastError();
        if (!src_on_device) {
            if (su3_d) (void)hipFree(su3_d);
            if (th_d) (void)hipFree(th_d);
        }
        if (partial) (void)hipFree(partial);
        free_gauge_dev(d);
        delete g;
    };
    if (!ok) {
        cleanup();
        return fail(CSTAR_ENOMEM, "cstar_gauge_create: device allocation failed");
    }
    hipError_t e = hipSuccess;
    if (!src_on_device) {
        e = hipMemcpyAsync(su3_d, su3, sizeof(double) * n_su3, hipMemcpyHostToDevice, g->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(th_d, theta, sizeof(double) * n_th, hipMemcpyHostToDevice, g->stream);
    } else {
        su3_d = const_cast<double *>(su3);
        th_d = const_cast<double *>(theta);
    }
    if (e == hipSuccess) e = launch_pack_links(g->geo, su3_d, th_d, par->q, d, g->stream);
    if (e == hipSuccess) e = launch_clover(g->geo, su3_d, th_d, par->q, par->csw_su3, par->csw_u1, d, partial, g->stream);
    std::vector<double> hp(clover_norm_blocks(g->geo));
    if (e == hipSuccess)
        e = hipMemcpyAsync(hp.data(), partial, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) {
        std::string msg = std::string("cstar_gauge_create: ") + hipGetErrorString(e);
        cleanup();
        return fail(CSTAR_EDEVICE, msg);
    }
    double nm = 0.0;
    for (double v : hp) nm = std::fmax(nm, v);
    g->clover_norm_max = nm;
    if (!src_on_device) {
        (void)hipFree(su3_d);
        (void)hipFree(th_d);
    }
    (void)hipFree(partial);
    HandleExtra *ex = new (std::nothrow) HandleExtra();
    if (!ex || hipMalloc(&ex->masses.dev, sizeof(double) * 4096) != hipSuccess) {
        delete ex;
        free_gauge_dev(d);
        delete g;
        return fail(CSTAR_ENOMEM, "cstar_gauge_create: device allocation failed");
    }
    ex->masses.cap = 4096;
    g->nn = nullptr;
    g->extra = ex;
    *out = g;
    return CSTAR_OK;
}

void cstar_gauge_destroy(cstar_gauge *g) {
    if (!g) return;
    (void)hipStreamSynchronize(g->stream);
    timing_release(g);
    workspace_release(g);
    eo_release(g);
    if (g->extra) {
        HandleExtra *ex = (HandleExtra *)g->extra;
        if (ex->masses.dev) (void)hipFree(ex->masses.dev);
        delete ex;
    }
    free_gauge_dev(g->d);
    delete g;
}

size_t cstar_spinor_bytes(const cstar_gauge *g, cstar_prec prec) {
    if (!g) return 0;
    const size_t n = (size_t)n_cplx(g->geo);
    return prec == CSTAR_FP64 ? n * 16 : n * 8;
}

long cstar_n_sites(const cstar_gauge *g) { return g ? 4L * g->geo.Vh : 0; }

static cstar_status check_prec(cstar_prec p) {
    if (p != CSTAR_FP64 && p != CSTAR_FP32 && p != CSTAR_FP32_BF16LINKS) return fail(CSTAR_EINVAL, "bad precision");
    return CSTAR_OK;
}

cstar_status cstar_spinor_pack(cstar_gauge *g, cstar_prec prec, int nrhs, const void *canonical, void *native) {
    if (!g || !canonical || !native || nrhs < 1) return fail(CSTAR_EINVAL, "cstar_spinor_pack: bad argument");
    if (check_prec(prec)) return CSTAR_EINVAL;
    CSTAR_HIP(launch_pack_spinor(g->geo, prec, nrhs, const_cast<void *>(canonical), native, 0, g->stream));
    return CSTAR_OK;
}

cstar_status cstar_spinor_unpack(cstar_gauge *g, cstar_prec prec, int nrhs, const void *native, void *canonical) {
    if (!g || !canonical || !native || nrhs < 1) return fail(CSTAR_EINVAL, "cstar_spinor_unpack: bad argument");
    if (check_prec(prec)) return CSTAR_EINVAL;
    CSTAR_HIP(launch_pack_spinor(g->geo, prec, nrhs, canonical, const_cast<void *>(native), 1, g->stream));
    return CSTAR_OK;
}

cstar_status dirac_apply(cstar_gauge *g, int nrhs, const double *masses, cstar_prec prec, int gamma5, const void *in,
                         void *out) {
    if (!g || !masses || !in || !out || nrhs < 1) return fail(CSTAR_EINVAL, "dirac_apply: bad argument");
    if (check_prec(prec)) return CSTAR_EINVAL;
    HandleExtra *ex = (HandleExtra *)g->extra;
    if (nrhs > ex->masses.cap) return fail(CSTAR_EINVAL, "dirac_apply: nrhs too large");
    bool same = true;
    for (int j = 0; j < nrhs; j++) {
        if (!std::isfinite(masses[j])) return fail(CSTAR_EINVAL, "dirac_apply: non-finite mass");
        if (masses[j] != masses[0]) same = false;
    }
    const size_t bytes = cstar_spinor_bytes(g, prec);
    const char *ib = (const char *)in, *ob = (const char *)out;
    if (ib < ob + bytes * nrhs && ob < ib + bytes * nrhs) return fail(CSTAR_EINVAL, "dirac_apply: in and out overlap");
    ApplyArgs a{in, out, (long)bytes, nrhs, gamma5 ? 1 : 0, nullptr, masses[0]};
    if (!same) {
        CSTAR_HIP(hipMemcpyAsync(ex->masses.dev, masses, sizeof(double) * nrhs, hipMemcpyHostToDevice, g->stream));
        a.masses_dev = ex->masses.dev;
    }
    CSTAR_HIP(handle_apply(g, prec, a));
    return CSTAR_OK;
}

}  // extern "C"

namespace {
// The learned preconditioner is optional: if the preconditioned solve fails
// (no convergence or a non-finite result) the plain solver answers.
cstar_status solve_with_fallback(cstar_gauge *g, double m0, int k, const cstar_eig_opts *opts, double *evals,
                                 double *resid, void *evecs, cstar_eig_stats *stats) {
    cstar_eig_stats st1{};
    cstar_status s = eig_lowest(g, m0, k, opts, evals, resid, evecs, &st1);
    bool bad = s != CSTAR_OK && s != CSTAR_EINVAL;
    if (s == CSTAR_OK)
        for (int i = 0; i < k; i++) bad = bad || !std::isfinite(evals[i]);
    if (opts && opts->use_nn && g->nn && bad) {
        cstar_eig_opts plain = *opts;
        plain.use_nn = 0;
        plain.warm_start = 0;
        cstar_eig_stats st2{};
        s = eig_lowest(g, m0, k, &plain, evals, resid, evecs, &st2);
        st2.applies_fp64 += st1.applies_fp64;
        st2.applies_inner += st1.applies_inner;
        st2.seconds += st1.seconds;
        st2.nn_applies = st1.nn_applies;
        st2.nn_fallback = 1;
        st1 = st2;
    }
    if (stats) *stats = st1;
    return s;
}
}  // namespace

extern "C" {

cstar_status q_lowest_eigs(cstar_gauge *g, double m0, int k, const cstar_eig_opts *opts, double *evals, double *resid,
                           void *evecs, cstar_eig_stats *stats) {
    if (!g || !evals || !std::isfinite(m0)) return fail(CSTAR_EINVAL, "q_lowest_eigs: bad argument");
    if (opts && check_prec(opts->inner)) return CSTAR_EINVAL;
    return solve_with_fallback(g, m0, k, opts, evals, resid, evecs, stats);
}

namespace {
struct GpuProvider {
    cstar_gauge *g;
    cstar_eig_opts opts;
    long applies = 0, nn_applies = 0;
    int fallbacks = 0;
    cstar_status last = CSTAR_OK;
    double lbar_tol = 1e-3;
    int lbar_calls = 0;
};
// lambda_bar for step A by the power method on Q^-2 (q_lambda_bar_power)
int gpu_lbar(void *ctx, double m, double *lb, double *err) {
    GpuProvider *p = (GpuProvider *)ctx;
    cstar_lbar_opts lo{};
    lo.tol = p->lbar_tol;
    lo.inner = p->opts.inner;  // the sign's precision: FP64 stays FP64, the mixed forms solve loose CGs in FP32
    cstar_lbar_stats st{};
    cstar_status s = q_lambda_bar_power(p->g, m, &lo, lb, err, &st);
    p->applies += st.applies_fp64 + st.applies_inner;
    p->lbar_calls++;
    p->last = s;
    return s == CSTAR_OK ? 0 : 1;
}
int gpu_provider(void *ctx, double m, int k, double *evals, double *errs) {
    GpuProvider *p = (GpuProvider *)ctx;
    cstar_eig_stats st{};
    cstar_status s = solve_with_fallback(p->g, m, k, &p->opts, evals, errs, nullptr, &st);
    p->applies += st.applies_fp64 + st.applies_inner;
    p->nn_applies += st.nn_applies;
    p->fallbacks += st.nn_fallback;
    p->last = s;
    // later points start from this point's Ritz block: the flow is followed in mass
    p->opts.warm_start = 1;
    return s == CSTAR_OK ? 0 : 1;
}
}  // namespace

cstar_status pfaffian_sign(cstar_gauge *g, const double *m_path, int n, const cstar_sign_opts *opts, int *sign_out,
                           cstar_sign_report *report) {
    if (!g || !m_path || !sign_out || n < 1 || !opts) return fail(CSTAR_EINVAL, "pfaffian_sign: bad argument");
    if (check_prec(opts->eig.inner)) return CSTAR_EINVAL;
    GpuProvider prov{g, opts->eig};
    prov.opts.warm_start = 0;
    const double c = opts->c > 0 ? opts->c : 1.9;
    // no eigenvalue of Q(m) vanishes for m > max_x ||SW(x)|| (the Wilson part has
    // non-negative Hermitian part); the margin keeps the top point off the bound
    const double m_max = opts->m_max > 0 ? opts->m_max : g->clover_norm_max * 1.001 + 1e-3;
    const int k = opts->k > 0 ? opts->k : 4;
    prov.lbar_tol = opts->lbar_tol > 0 ? opts->lbar_tol : 1e-3;
    cstar_status st = opts->step_a_power
                          ? sign_driver_stepa(gpu_lbar, gpu_provider, &prov, m_path, n, k, c, m_max, sign_out, report)
                          : sign_driver(gpu_provider, &prov, m_path, n, k, c, m_max, sign_out, report);
    if (report) {
        report->applies = prov.applies;
        report->nn_applies = prov.nn_applies;
        report->nn_fallbacks = prov.fallbacks;
    }
    if (st == CSTAR_ENOCONV && prov.last != CSTAR_OK) return prov.last;
    return st;
}

cstar_status cstar_sign_driver(cstar_eig_provider provider, void *ctx, const double *m_path, int n, int k, double c,
                               double m_max, int *sign_out, cstar_sign_report *report) {
    return sign_driver(provider, ctx, m_path, n, k, c, m_max, sign_out, report);
}

cstar_status cstar_sign_driver_a(cstar_lbar_provider lbar, cstar_eig_provider provider, void *ctx,
                                 const double *m_path, int n, int k, double c, double m_max, int *sign_out,
                                 cstar_sign_report *report) {
    return sign_driver_stepa(lbar, provider, ctx, m_path, n, k, c, m_max, sign_out, report);
}

cstar_status cstar_clover_norm_max(cstar_gauge *g, double *out) {
    if (!g || !out) return fail(CSTAR_EINVAL, "cstar_clover_norm_max: bad argument");
    *out = g->clover_norm_max;
    return CSTAR_OK;
}

}  // extern "C"
