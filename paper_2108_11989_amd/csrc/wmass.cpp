// Mass-reweighting factor W_mass by its stochastic estimator (C ABI in include/cstar.h).
//
// Paper, mass-reweighting section: with R(x) = A prod_i (x + nu_i^2)/(x + mu_i^2)
// approximating x^{-1/4}, W_mass = det[R(Q_hat_m^2) R^{-1}(Q_hat_m'^2)] factorises
// over the rational factors i into determinants of positive Hermitian
// operators built from delta D_hat = D_hat_m' - D_hat_m and
//   S_i = (D_hat_m + i g5 nu_i)^{-1} - (D_hat_m' + i g5 mu_i)^{-1}
//         - (D_hat_m' + i g5 mu_i)^{-1} delta D_hat (D_hat_m + i g5 nu_i)^{-1},
// each estimated with Gaussian sources eta on the even sites:
//   W_i ~ (1/N) sum_l exp(-(eta_l, R_i eta_l)),
//   R_i = (dD S_i)^H + dD S_i + (dD S_i)^H (dD S_i) = (1 + dD S_i)^H (1 + dD S_i) - 1.
// (The Gaussian average of exp(-(eta, R eta)) is det(1 + R)^{-1}; with the S_i
// above, det(1 + R_i)^{-1} is the i-th factor of det[R(Q_hat_m^2) R^{-1}(Q_hat_m'^2)].)
//
// S_i = B^{-1} (B - A - dD) A^{-1} = B^{-1} i g5 (mu_i - nu_i) A^{-1} with A = D_hat_m + i g5 nu_i,
// B = D_hat_m' + i g5 mu_i, and (D_hat + i g5 s)^{-1} = (Q_hat - i s)(Q_hat^2 + s^2)^{-1} g5:
// every inverse is one solve of Q_hat^2 + s^2 to relative FP64 residual tol
// and one application of Q_hat, on the library's even-odd operator.  The
// solve is mixed-precision iterative refinement: FP32 conjugate gradients on
// the FP32-row operator reduce the FP64 residual r = b - (Q_hat^2 + s^2) x by
// 1e-5 per round (x += e), until ||r|| <= tol ||b||; a round that gains less
// than a factor 2 hands the rest to FP64 CG.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "blas.h"
#include "cstar_internal.h"

namespace cstar {
namespace {

struct Ctx {
    cstar_gauge *g;
    long ne;      // complex entries of an even FP64 vector
    double2 *partial = nullptr, *dotdev = nullptr;
    long cg_iters = 0, applies = 0;
    // FP32 refinement: CG vectors (even, FP32 native) and two FP64 even vectors
    float4 *r32 = nullptr, *p32 = nullptr, *ap32 = nullptr, *tmp32 = nullptr, *x32 = nullptr;
    double2 *e = nullptr, *e2 = nullptr;
};

cstar_status dot(Ctx &c, const double2 *u, const double2 *v, double2 *out) {
    CSTAR_HIP(launch_gram(u, c.ne, 1, v, c.ne, 1, c.ne, c.partial, c.dotdev, c.g->stream));
    CSTAR_HIP(hipMemcpyAsync(out, c.dotdev, sizeof(double2), hipMemcpyDeviceToHost, c.g->stream));
    CSTAR_HIP(hipStreamSynchronize(c.g->stream));
    return CSTAR_OK;
}

// out = (Q_hat(m)^2 + sigma) in   (tmp: one even vector)
cstar_status q2s(Ctx &c, double m, double sigma, const double2 *in, double2 *out, double2 *tmp) {
    cstar_status st = eo_apply(c.g, 1, m, CSTAR_FP64, 1, in, tmp);
    if (!st) st = eo_apply(c.g, 1, m, CSTAR_FP64, 1, tmp, out);
    if (st) return st;
    c.applies += 2;
    CSTAR_HIP(launch_lincomb64(2 * c.ne, sigma, (const double *)in, 1.0, (double *)out, 0.0, nullptr, c.g->stream));
    return CSTAR_OK;
}

cstar_status dot32(Ctx &c, const float4 *u, const float4 *v, double *out) {
    CSTAR_HIP(launch_dot32(u, v, c.ne / 2, c.partial, c.dotdev, c.g->stream));
    double2 h;
    CSTAR_HIP(hipMemcpyAsync(&h, c.dotdev, sizeof(double2), hipMemcpyDeviceToHost, c.g->stream));
    CSTAR_HIP(hipStreamSynchronize(c.g->stream));
    *out = h.x;
    return CSTAR_OK;
}

// out = (Q_hat(m)^2 + sigma) in on the FP32-row operator (tmp: one FP32 even vector)
cstar_status q2s32(Ctx &c, double m, double sigma, const float4 *in, float4 *out, float4 *tmp) {
    cstar_status st = eo_apply(c.g, 1, m, CSTAR_FP32, 1, in, tmp);
    if (!st) st = eo_apply(c.g, 1, m, CSTAR_FP32, 1, tmp, out);
    if (st) return st;
    c.applies += 2;
    CSTAR_HIP(launch_lincomb32(2 * c.ne, (float)sigma, (const float *)in, 1.f, (float *)out, 0.f, nullptr,
                               c.g->stream));
    return CSTAR_OK;
}

// x32 = (Q_hat(m)^2 + sigma)^{-1} r32 in FP32 arithmetic, until the FP32
// residual (r32, overwritten) falls below tol of its start
cstar_status cg32(Ctx &c, double m, double sigma, double tol, int maxit) {
    hipStream_t s = c.g->stream;
    const size_t bytes = (size_t)(c.ne / 2) * sizeof(float4);
    CSTAR_HIP(hipMemsetAsync(c.x32, 0, bytes, s));
    CSTAR_HIP(hipMemcpyAsync(c.p32, c.r32, bytes, hipMemcpyDeviceToDevice, s));
    double rr;
    cstar_status st = dot32(c, c.r32, c.r32, &rr);
    if (st) return st;
    const double stop = tol * tol * rr;
    for (int it = 0; it < maxit && rr > stop; it++) {
        st = q2s32(c, m, sigma, c.p32, c.ap32, c.tmp32);
        double pap;
        if (!st) st = dot32(c, c.p32, c.ap32, &pap);
        if (st) return st;
        if (!(pap > 0.0)) break;
        const double a = rr / pap;
        CSTAR_HIP(launch_lincomb32(2 * c.ne, (float)a, (const float *)c.p32, 1.f, (float *)c.x32, 0.f, nullptr, s));
        CSTAR_HIP(launch_lincomb32(2 * c.ne, (float)-a, (const float *)c.ap32, 1.f, (float *)c.r32, 0.f, nullptr, s));
        double rn;
        if ((st = dot32(c, c.r32, c.r32, &rn))) return st;
        c.cg_iters++;
        CSTAR_HIP(launch_lincomb32(2 * c.ne, 1.f, (const float *)c.r32, (float)(rn / rr), (float *)c.p32, 0.f, nullptr,
                                   s));
        rr = rn;
    }
    return CSTAR_OK;
}

// x = (Q_hat(m)^2 + sigma)^{-1} b by CG from x = 0, until ||r|| <= tol ||b||.
cstar_status cg(Ctx &c, double m, double sigma, const double2 *b, double2 *x, double2 *r, double2 *p, double2 *ap,
                double2 *tmp, double tol, int maxit) {
    const size_t bytes = sizeof(double2) * c.ne;
    hipStream_t s = c.g->stream;
    CSTAR_HIP(hipMemsetAsync(x, 0, bytes, s));
    CSTAR_HIP(hipMemcpyAsync(r, b, bytes, hipMemcpyDeviceToDevice, s));
    CSTAR_HIP(hipMemcpyAsync(p, b, bytes, hipMemcpyDeviceToDevice, s));
    double2 d;
    cstar_status st = dot(c, r, r, &d);
    if (st) return st;
    double rr = d.x;
    const double stop = tol * tol * rr;
    if (rr == 0.0) return CSTAR_OK;
    for (int it = 0; it < maxit; it++) {
        st = q2s(c, m, sigma, p, ap, tmp);
        if (!st) st = dot(c, p, ap, &d);
        if (st) return st;
        const double alpha = rr / d.x;
        CSTAR_HIP(launch_lincomb64(2 * c.ne, alpha, (const double *)p, 1.0, (double *)x, 0.0, nullptr, s));
        CSTAR_HIP(launch_lincomb64(2 * c.ne, -alpha, (const double *)ap, 1.0, (double *)r, 0.0, nullptr, s));
        st = dot(c, r, r, &d);
        if (st) return st;
        c.cg_iters++;
        if (d.x <= stop) return CSTAR_OK;
        const double beta = d.x / rr;
        rr = d.x;
        CSTAR_HIP(launch_lincomb64(2 * c.ne, 1.0, (const double *)r, beta, (double *)p, 0.0, nullptr, s));
    }
    return fail(CSTAR_ENOCONV, "cstar_w_mass: conjugate gradient did not reach the tolerance");
}

// the same solve by mixed-precision iterative refinement (file header)
cstar_status cg_mixed(Ctx &c, double m, double sigma, const double2 *b, double2 *x, double2 *r, double2 *p,
                      double2 *ap, double2 *tmp, double tol, int maxit) {
    const size_t bytes = sizeof(double2) * c.ne;
    hipStream_t s = c.g->stream;
    CSTAR_HIP(hipMemsetAsync(x, 0, bytes, s));
    CSTAR_HIP(hipMemcpyAsync(r, b, bytes, hipMemcpyDeviceToDevice, s));
    double2 d;
    cstar_status st = dot(c, b, b, &d);
    if (st) return st;
    const double bb = d.x;
    double rr = bb;
    if (bb == 0.0) return CSTAR_OK;
    for (int round = 0; round < 40; round++) {
        CSTAR_HIP(launch_even_to_f32(c.g->geo, r, c.r32, s));
        if ((st = cg32(c, m, sigma, 1e-5, maxit))) return st;
        CSTAR_HIP(launch_even_to_f64(c.g->geo, c.x32, c.e, s));
        CSTAR_HIP(launch_lincomb64(2 * c.ne, 1.0, (const double *)c.e, 1.0, (double *)x, 0.0, nullptr, s));
        // r = b - (Q_hat^2 + sigma) x in FP64
        if ((st = q2s(c, m, sigma, x, ap, tmp))) return st;
        CSTAR_HIP(launch_lincomb64(2 * c.ne, -1.0, (const double *)ap, 0.0, (double *)r, 1.0, (const double *)b, s));
        if ((st = dot(c, r, r, &d))) return st;
        const double rn = d.x;
        if (rn <= tol * tol * bb) return CSTAR_OK;
        if (!(rn <= 0.25 * rr)) {
            // FP32 has stopped gaining: the rest in FP64, x += (Q_hat^2 + sigma)^{-1} r
            CSTAR_HIP(hipMemcpyAsync(c.e2, r, bytes, hipMemcpyDeviceToDevice, s));
            if ((st = cg(c, m, sigma, c.e2, c.e, r, p, ap, tmp, std::min(1.0, tol * std::sqrt(bb / rn)), maxit)))
                return st;
            CSTAR_HIP(launch_lincomb64(2 * c.ne, 1.0, (const double *)c.e, 1.0, (double *)x, 0.0, nullptr, s));
            return CSTAR_OK;
        }
        rr = rn;
    }
    return fail(CSTAR_ENOCONV, "cstar_w_mass: iterative refinement did not reach the tolerance");
}

// out = (D_hat(m) + i g5 s)^{-1} in = (Q_hat - i s)(Q_hat^2 + s^2)^{-1} g5 in
cstar_status shifted_inverse(Ctx &c, double m, double s, const double2 *in, double2 *out, double2 *w[6], double tol,
                             int maxit) {
    double2 *g5in = w[0], *y = w[1];
    hipStream_t st_ = c.g->stream;
    CSTAR_HIP(hipMemsetAsync(g5in, 0, sizeof(double2) * c.ne, st_));
    CSTAR_HIP(launch_even_axpy(c.g->geo, 1.0, 0.0, 1, in, g5in, st_));
    cstar_status st = cg_mixed(c, m, s * s, g5in, y, w[2], w[3], w[4], w[5], tol, maxit);
    if (!st) st = eo_apply(c.g, 1, m, CSTAR_FP64, 1, y, out);
    if (st) return st;
    c.applies++;
    CSTAR_HIP(launch_even_axpy(c.g->geo, 0.0, -s, 0, y, out, st_));
    return CSTAR_OK;
}

}  // namespace
}  // namespace cstar

using namespace cstar;

extern "C" cstar_status cstar_w_mass(cstar_gauge *g, double m, double m_prime, int n, const double *nu2,
                                     const double *mu2, int nsrc, const void *eta, double tol, double *expo,
                                     double *log_w_mass, cstar_wmass_stats *stats) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!g || !nu2 || !mu2 || !eta || !expo || !log_w_mass || n < 1 || nsrc < 1 || !std::isfinite(m) ||
        !std::isfinite(m_prime) || !(tol > 0))
        return fail(CSTAR_EINVAL, "cstar_w_mass: bad argument");
    for (int i = 0; i < n; i++)
        if (!(nu2[i] >= 0) || !(mu2[i] >= 0) || !std::isfinite(nu2[i]) || !std::isfinite(mu2[i]))
            return fail(CSTAR_EINVAL, "cstar_w_mass: shifts must be finite and non-negative");
    Ctx c{g, 24L * g->geo.Vh};
    const size_t vb = sizeof(double2) * c.ne;
    const int NV = 13;
    double2 *buf = nullptr;
    if (hipMalloc(&buf, vb * NV) != hipSuccess || hipMalloc(&c.partial, gram_partial_bytes()) != hipSuccess ||
        hipMalloc(&c.dotdev, sizeof(double2)) != hipSuccess) {
        (void)hipGetLastError();
        if (buf) (void)hipFree(buf);
        if (c.partial) (void)hipFree(c.partial);
        return fail(CSTAR_ENOMEM, "cstar_w_mass: device allocation failed");
    }
    double2 *a = buf, *w2 = buf + c.ne, *bv = buf + 2 * c.ne, *u = buf + 3 * c.ne, *u2 = buf + 4 * c.ne;
    double2 *w[6];
    for (int k = 0; k < 6; k++) w[k] = buf + (5 + k) * c.ne;
    c.e = buf + 11 * c.ne;
    c.e2 = buf + 12 * c.ne;
    float4 *buf32 = nullptr;
    if (hipMalloc(&buf32, sizeof(float4) * (c.ne / 2) * 5) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(buf);
        (void)hipFree(c.partial);
        (void)hipFree(c.dotdev);
        return fail(CSTAR_ENOMEM, "cstar_w_mass: device allocation failed");
    }
    c.r32 = buf32;
    c.p32 = buf32 + c.ne / 2;
    c.ap32 = buf32 + 2 * (c.ne / 2);
    c.tmp32 = buf32 + 3 * (c.ne / 2);
    c.x32 = buf32 + 4 * (c.ne / 2);
    hipStream_t s = g->stream;
    const int maxit = 100000;
    cstar_status st = CSTAR_OK;
    for (int l = 0; l < nsrc && !st; l++) {
        const double2 *el = (const double2 *)eta + (long)l * c.ne;
        double2 d;
        st = dot(c, el, el, &d);
        const double ee = d.x;
        for (int i = 0; i < n && !st; i++) {
            const double nu = std::sqrt(nu2[i]), mu = std::sqrt(mu2[i]);
            // a = (D_hat_m + i g5 nu)^{-1} eta;  w2 = i g5 (mu - nu) a;  bv = (D_hat_m' + i g5 mu)^{-1} w2 = S_i eta
            st = shifted_inverse(c, m, nu, el, a, w, tol, maxit);
            if (st) break;
            if (hipMemsetAsync(w2, 0, vb, s) != hipSuccess ||
                launch_even_axpy(g->geo, 0.0, mu - nu, 1, a, w2, s) != hipSuccess) {
                st = fail(CSTAR_EDEVICE, "cstar_w_mass: kernel launch failed");
                break;
            }
            st = shifted_inverse(c, m_prime, mu, w2, bv, w, tol, maxit);
            // u = eta + (D_hat_m' - D_hat_m) bv; (eta, R_i eta) = |u|^2 - |eta|^2
            if (!st) st = eo_apply(g, 1, m_prime, CSTAR_FP64, 0, bv, u);
            if (!st) st = eo_apply(g, 1, m, CSTAR_FP64, 0, bv, u2);
            if (st) break;
            c.applies += 2;
            if (launch_lincomb64(2 * c.ne, -1.0, (const double *)u2, 1.0, (double *)u, 1.0, (const double *)el, s) !=
                hipSuccess) {
                st = fail(CSTAR_EDEVICE, "cstar_w_mass: kernel launch failed");
                break;
            }
            st = dot(c, u, u, &d);
            expo[(long)i * nsrc + l] = d.x - ee;
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipFree(buf);
    (void)hipFree(buf32);
    (void)hipFree(c.partial);
    (void)hipFree(c.dotdev);
    if (st) return st;
    // log W_mass = sum_i log((1/N) sum_l exp(-x_il)), by log-sum-exp
    double lw = 0.0;
    for (int i = 0; i < n; i++) {
        double mn = 1e300;
        for (int l = 0; l < nsrc; l++) mn = std::fmin(mn, expo[(long)i * nsrc + l]);
        double acc = 0.0;
        for (int l = 0; l < nsrc; l++) acc += std::exp(-(expo[(long)i * nsrc + l] - mn));
        lw += -mn + std::log(acc / nsrc);
    }
    *log_w_mass = lw;
    if (stats) {
        stats->cg_iterations = c.cg_iters;
        stats->eo_applies = c.applies;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return CSTAR_OK;
}
