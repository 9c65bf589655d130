// lambda_bar(m) = min |lambda(Q(m))| by the power method with Chebyshev
// acceleration on B = Q(m)^-2 (the paper's choice for step A of the sign
// algorithm, Sec. 3: only the smallest |eigenvalue| is needed, no eigenvector
// is tracked).  Every product B y is a conjugate-gradient solve of
// Q^2 x = y in FP64 on the library's apply and vector kernels.
//
//   * a few plain power steps v <- B v / |B v|;
//   * then steps v <- T_d(2 B / beta - 1) v / |.|, the Chebyshev polynomial
//     that is bounded by 1 on the unwanted part [0, beta] of B's spectrum and
//     grows fastest above it; beta starts from the contraction of the plain
//     steps and is raised to the second eigenvalue of B implied by each
//     Chebyshev step's observed contraction (adaptive Chebyshev iteration,
//     Manteuffel, Numer. Math. 28 (1977)), never above 0.98 of the current
//     estimate of the first;
//   * the convergence test uses the exact Q^2 residual: theta = v^H Q^2 v,
//     r = |Q^2 v - theta v|; some eigenvalue of Q^2 lies in [theta - r,
//     theta + r], so sqrt(theta) carries the half-width
//     max(sqrt(theta) - sqrt(theta - r), sqrt(theta + r) - sqrt(theta));
//     theta itself is an upper bound of lambda_bar^2 (Rayleigh quotient).
// The inner solves are inexact on purpose: their tolerance follows the outer
// residual (0.01 of it, within [1e-13, 1e-3]), which slows the outer
// iteration but cannot bias the reported bound.  For the same reason a solve
// whose tolerance is 1e-6 or looser may run in FP32 arithmetic (opts.inner)
// on the operator with FP32 link rows, whose difference from the FP64 one
// (~1e-7 relative) is far below those tolerances -- BF16 rows (~4e-3) would
// move the eigenvector the iteration converges to, so an FP32 request of
// either form uses FP32 rows; the tighter solves, and every Rayleigh quotient
// and residual, stay in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "blas.h"
#include "cstar_internal.h"

namespace cstar {
namespace {

struct Power {
    cstar_gauge *g;
    hipStream_t s;
    double m;
    long n;  // complex entries per FP64 vector
    cstar_prec inner = CSTAR_FP64;
    double2 *partial = nullptr, *gout = nullptr;
    float4 *r32 = nullptr, *p32 = nullptr, *ap32 = nullptr, *tmp32 = nullptr, *x32 = nullptr;  // FP32 inner CG
    double2 *e = nullptr;   // FP64 correction of an FP32 solution
    bool fp32_off = false;  // set once an FP32 solve missed its tolerance: FP64 from then on
    long applies = 0, applies_inner = 0, cg_iterations = 0;
    int solves = 0;
    std::vector<void *> owned;

    ~Power() {
        for (void *p : owned) (void)hipFree(p);
    }
    template <class T>
    cstar_status alloc(T **p, size_t bytes) {
        if (hipMalloc((void **)p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(CSTAR_ENOMEM, "q_lambda_bar_power: device allocation failed");
        }
        owned.push_back(*p);
        return CSTAR_OK;
    }
    // out = Q(m)^2 in, through tmp
    cstar_status q2(const double2 *in, double2 *tmp, double2 *out) {
        const long st = n * (long)sizeof(double2);
        ApplyArgs a{in, tmp, st, 1, 1, nullptr, m};
        CSTAR_HIP(handle_apply(g, CSTAR_FP64, a));
        ApplyArgs b{tmp, out, st, 1, 1, nullptr, m};
        CSTAR_HIP(handle_apply(g, CSTAR_FP64, b));
        applies += 2;
        return CSTAR_OK;
    }
    // real part of x^H y (host value; synchronises the stream)
    cstar_status dot(const double2 *x, const double2 *y, double *out) {
        CSTAR_HIP(launch_gram(x, n, 1, y, n, 1, n, partial, gout, s));
        double2 h;
        CSTAR_HIP(hipMemcpyAsync(&h, gout, sizeof(double2), hipMemcpyDeviceToHost, s));
        CSTAR_HIP(hipStreamSynchronize(s));
        *out = h.x;
        return CSTAR_OK;
    }
    // y = a x + b y (+ c z)
    cstar_status lin(double a, const double2 *x, double b, double2 *y, double c = 0.0, const double2 *z = nullptr) {
        CSTAR_HIP(launch_lincomb64(2 * n, a, (const double *)x, b, (double *)y, c, (const double *)z, s));
        return CSTAR_OK;
    }
    // y = a y through the lincomb kernel with x = y: every element is read and
    // then written by the same lane, nothing else touches it (the kernel's
    // restrict qualifiers are formally violated by this call, harmlessly)
    cstar_status scale(double2 *y, double a) { return lin(0.0, y, a, y); }
    cstar_status copy(const double2 *x, double2 *y) {
        if (x == y) return CSTAR_OK;
        CSTAR_HIP(hipMemcpyAsync(y, x, sizeof(double2) * n, hipMemcpyDeviceToDevice, s));
        return CSTAR_OK;
    }

    // out = Q(m)^2 in, in the FP32 form `inner`, through tmp
    cstar_status q2f(const float4 *in, float4 *tmp, float4 *out) {
        const long st = n / 2 * (long)sizeof(float4);
        ApplyArgs a{in, tmp, st, 1, 1, nullptr, m};
        CSTAR_HIP(handle_apply(g, inner, a));
        ApplyArgs b{tmp, out, st, 1, 1, nullptr, m};
        CSTAR_HIP(handle_apply(g, inner, b));
        applies_inner += 2;
        return CSTAR_OK;
    }
    cstar_status dot32(const float4 *x, const float4 *y, double *out) {
        CSTAR_HIP(launch_dot32(x, y, n / 2, partial, gout, s));
        double2 h;
        CSTAR_HIP(hipMemcpyAsync(&h, gout, sizeof(double2), hipMemcpyDeviceToHost, s));
        CSTAR_HIP(hipStreamSynchronize(s));
        *out = h.x;
        return CSTAR_OK;
    }
    cstar_status lin32(float a, const float4 *x, float b, float4 *y) {
        CSTAR_HIP(launch_lincomb32(2 * n, a, (const float *)x, b, (float *)y, 0.f, nullptr, s));
        return CSTAR_OK;
    }
    // x = (Q^2)^-1 b as solve() below, in FP32 arithmetic on the FP32 form
    // `inner` (b and x FP64, converted on the way in and out)
    cstar_status solve32(const double2 *b, double2 *x, double tol, int maxit) {
        const size_t bytes = (size_t)(n / 2) * sizeof(float4);
        CSTAR_HIP(launch_to_f32(g->geo, 1, b, r32, s));
        CSTAR_HIP(hipMemcpyAsync(p32, r32, bytes, hipMemcpyDeviceToDevice, s));
        CSTAR_HIP(hipMemsetAsync(x32, 0, bytes, s));
        cstar_status st;
        double rr;
        if ((st = dot32(r32, r32, &rr))) return st;
        const double stop = tol * tol * rr;
        solves++;
        for (int it = 0; it < maxit && rr > stop; it++) {
            if ((st = q2f(p32, tmp32, ap32))) return st;
            double pap;
            if ((st = dot32(p32, ap32, &pap))) return st;
            if (!(pap > 0.0)) break;
            const double a = rr / pap;
            if ((st = lin32((float)a, p32, 1.f, x32)) || (st = lin32((float)-a, ap32, 1.f, r32))) return st;
            double rn;
            if ((st = dot32(r32, r32, &rn))) return st;
            if ((st = lin32(1.f, r32, (float)(rn / rr), p32))) return st;
            rr = rn;
            cg_iterations++;
        }
        CSTAR_HIP(launch_to_f64(g->geo, 1, x32, x, s));
        return CSTAR_OK;
    }
    // x = (Q^2)^-1 b by CG from x = 0 to relative residual tol (at most maxit steps)
    cstar_status solve(const double2 *b, double2 *x, double2 *r, double2 *p, double2 *ap, double2 *tmp, double tol,
                       int maxit) {
        cstar_status st;
        CSTAR_HIP(hipMemsetAsync(x, 0, sizeof(double2) * n, s));
        if ((st = copy(b, r)) || (st = copy(b, p))) return st;
        double rr;
        if ((st = dot(r, r, &rr))) return st;
        const double stop = tol * tol * rr;
        solves++;
        for (int it = 0; it < maxit && rr > stop; it++) {
            if ((st = q2(p, tmp, ap))) return st;
            double pap;
            if ((st = dot(p, ap, &pap))) return st;
            if (!(pap > 0.0)) break;  // Q^2 is positive definite: only rounding ends here
            const double a = rr / pap;
            if ((st = lin(a, p, 1.0, x)) || (st = lin(-a, ap, 1.0, r))) return st;
            double rn;
            if ((st = dot(r, r, &rn))) return st;
            if ((st = lin(1.0, r, rn / rr, p))) return st;
            rr = rn;
            cg_iterations++;
        }
        return CSTAR_OK;
    }
    // the FP32 solve where the tolerance allows it.  FP32 CG's own residual
    // can fall below the tolerance while the true one stalls near FP32
    // rounding times the condition number of Q^2, so the solution's residual
    // is recomputed in FP64; if it misses the tolerance by more than 10x, an
    // FP64 solve of the correction finishes the job and every later solve is
    // FP64.
    cstar_status solve_any(const double2 *b, double2 *x, double2 *r, double2 *p, double2 *ap, double2 *tmp,
                           double tol, int maxit) {
        if (inner == CSTAR_FP64 || fp32_off || tol < 1e-6) return solve(b, x, r, p, ap, tmp, tol, maxit);
        cstar_status st;
        if ((st = solve32(b, x, tol, maxit))) return st;
        double rr, bb;
        if ((st = q2(x, tmp, ap)) || (st = copy(b, r)) || (st = lin(-1.0, ap, 1.0, r)) || (st = dot(r, r, &rr)) ||
            (st = dot(b, b, &bb)))
            return st;
        if (rr <= 100.0 * tol * tol * bb) return CSTAR_OK;
        fp32_off = true;
        if ((st = solve(r, e, r, p, ap, tmp, std::min(1.0, tol * std::sqrt(bb / rr)), maxit))) return st;
        return lin(1.0, e, 1.0, x);
    }
    // theta = v^H Q^2 v and r = |Q^2 v - theta v| for unit v (y, tmp: scratch)
    cstar_status residual(const double2 *v, double2 *y, double2 *tmp, double *theta, double *r) {
        cstar_status st;
        if ((st = q2(v, tmp, y)) || (st = dot(v, y, theta)) || (st = lin(-*theta, v, 1.0, y))) return st;
        double rr;
        if ((st = dot(y, y, &rr))) return st;
        *r = std::sqrt(std::max(rr, 0.0));
        return CSTAR_OK;
    }
    cstar_status normalise(double2 *v, double *norm = nullptr) {
        double vv;
        cstar_status st = dot(v, v, &vv);
        if (st) return st;
        if (!(vv > 0.0) || !std::isfinite(vv)) return fail(CSTAR_ENOCONV, "q_lambda_bar_power: vector vanished");
        if (norm) *norm = std::sqrt(vv);
        return scale(v, 1.0 / std::sqrt(vv));
    }
};

double half_width(double theta, double r) {
    const double s = std::sqrt(std::max(theta, 0.0));
    return std::max(s - std::sqrt(std::max(theta - r, 0.0)), std::sqrt(theta + r) - s);
}

}  // namespace
}  // namespace cstar

using namespace cstar;

extern "C" cstar_status q_lambda_bar_power(cstar_gauge *g, double m0, const cstar_lbar_opts *opts_in,
                                           double *lambda_bar, double *bound, cstar_lbar_stats *stats) {
    if (!g || !lambda_bar || !std::isfinite(m0)) return fail(CSTAR_EINVAL, "q_lambda_bar_power: bad argument");
    cstar_lbar_opts o{};
    if (opts_in) o = *opts_in;
    if (!(o.tol >= 0.0) || o.degree < 0 || o.degree > 64 || o.plain_steps < 0 || o.max_outer < 0 || o.max_cg < 0 ||
        (o.inner != CSTAR_FP64 && o.inner != CSTAR_FP32 && o.inner != CSTAR_FP32_BF16LINKS))
        return fail(CSTAR_EINVAL, "q_lambda_bar_power: bad options");
    const double tol = o.tol > 0.0 ? o.tol : 1e-3;
    const int deg = o.degree > 0 ? o.degree : 8;
    const int nplain = o.plain_steps > 0 ? o.plain_steps : 3;
    const int max_outer = o.max_outer > 0 ? o.max_outer : 500;
    const int max_cg = o.max_cg > 0 ? o.max_cg : 20000;
    const auto t0 = std::chrono::steady_clock::now();
    if (hipSetDevice(g->device) != hipSuccess) return fail(CSTAR_EDEVICE, "q_lambda_bar_power: hipSetDevice");

    Power P{g, g->stream, m0, n_cplx(g->geo), o.inner == CSTAR_FP64 ? CSTAR_FP64 : CSTAR_FP32};
    const size_t vb = sizeof(double2) * P.n;
    double2 *v, *x, *r, *p, *ap, *tmp, *y0, *y1;
    cstar_status st;
    for (double2 **b : {&v, &x, &r, &p, &ap, &tmp, &y0, &y1})
        if ((st = P.alloc(b, vb))) return st;
    if ((st = P.alloc(&P.partial, gram_partial_bytes())) || (st = P.alloc(&P.gout, sizeof(double2) * 64)))
        return st;
    if (P.inner != CSTAR_FP64) {
        for (float4 **b : {&P.r32, &P.p32, &P.ap32, &P.tmp32, &P.x32})
            if ((st = P.alloc(b, (size_t)(P.n / 2) * sizeof(float4)))) return st;
        if ((st = P.alloc(&P.e, vb))) return st;
    }

    CSTAR_HIP(launch_gauss(v, P.n, o.seed, P.s));
    if ((st = P.normalise(v))) return st;
    double theta, res;
    if ((st = P.residual(v, y0, tmp, &theta, &res))) return st;
    double rel = res / theta, rel_prev = rel;
    double beta = 0.0;  // 0: plain power steps
    int outer = 0;
    bool conv = half_width(theta, res) <= tol * std::sqrt(theta);
    while (!conv && outer < max_outer) {
        const double tin = std::max(1e-13, std::min(1e-3, 0.01 * rel));
        if (beta <= 0.0) {
            if ((st = P.solve_any(v, x, r, p, ap, tmp, tin, max_cg)) || (st = P.copy(x, v))) return st;
        } else {
            // T_d(2B/beta - 1) v: y_1 = (2/beta) B v - v, y_{k+1} = (4/beta) B y_k - 2 y_k - y_{k-1},
            // the pair rescaled together after every step (only the direction matters)
            if ((st = P.copy(v, y0)) || (st = P.solve_any(v, x, r, p, ap, tmp, tin, max_cg)) || (st = P.copy(x, y1)) ||
                (st = P.lin(-1.0, v, 2.0 / beta, y1)))
                return st;
            for (int k = 1; k < deg; k++) {
                if ((st = P.solve_any(y1, x, r, p, ap, tmp, tin, max_cg)) ||
                    (st = P.lin(4.0 / beta, x, -1.0, y0, -2.0, y1)))
                    return st;
                double nrm;
                if ((st = P.normalise(y0, &nrm)) || (st = P.scale(y1, 1.0 / nrm))) return st;
                std::swap(y0, y1);
            }
            if ((st = P.copy(y1, v))) return st;
        }
        if ((st = P.normalise(v)) || (st = P.residual(v, y0, tmp, &theta, &res))) return st;
        outer++;
        rel_prev = rel;
        rel = res / theta;
        conv = half_width(theta, res) <= tol * std::sqrt(theta);
        const double mu1 = 1.0 / theta;
        if (beta <= 0.0) {
            if (outer >= nplain) beta = std::min(0.9, std::max(0.02, rel / rel_prev)) * mu1;
        } else {
            // contraction k of this step = T_d(x2) / T_d(x1) with x_i = 2 mu_i / beta - 1 -> mu2
            const double kobs = std::min(rel / rel_prev, 0.999);
            const double x1 = 2.0 * mu1 / beta - 1.0;
            const double arg = kobs * std::cosh(deg * std::acosh(std::max(x1, 1.0)));
            const double mu2 = 0.5 * beta * (1.0 + (arg > 1.0 ? std::cosh(std::acosh(arg) / deg) : 1.0));
            beta = std::min(0.98 * mu1, std::max(beta, mu2));
        }
    }
    *lambda_bar = std::sqrt(theta);
    if (bound) *bound = half_width(theta, res);
    if (stats) {
        stats->outer = outer;
        stats->solves = P.solves;
        stats->cg_iterations = P.cg_iterations;
        stats->applies_fp64 = P.applies;
        stats->applies_inner = P.applies_inner;
        stats->beta = beta;
        stats->resid_q2 = res;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (!conv) return fail(CSTAR_ENOCONV, "q_lambda_bar_power: max_outer reached before tol");
    return CSTAR_OK;
}
