// Rational approximation of x^{-1/4} for the mass-reweighting factor (C ABI in include/cstar.h).
//
// Paper, mass-reweighting section (eq. ratapprox): (Q_hat^2)^{-1/4} is
// replaced by R(Q_hat^2), R(x) = A prod_{i=1}^n (x + nu_i^2) / (x + mu_i^2), the
// optimal approximation of order (n, n) on [r_a, r_b] in the sense of the
// smallest uniform relative error.  The relative error is measured as
// e(x) = log(R(x) x^{1/4}) (equal to R(x) x^{1/4} - 1 to first order), and the
// minimax R is found by the Remez exchange: on a reference of 2n+2 points e
// takes the values +-delta with alternating signs (Newton's method on log A,
// log nu_i^2, log mu_i^2 and delta), then the reference moves to the 2n+2
// alternating extrema of e on [r_a, r_b], until their moduli agree.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "cstar_internal.h"

namespace cstar {
namespace {

struct Rat {
    int n;
    double logA;
    std::vector<double> lz, lp;  // log nu^2, log mu^2
    double err(double x) const {
        double v = logA + 0.25 * std::log(x);
        for (int i = 0; i < n; i++) v += std::log(x + std::exp(lz[i])) - std::log(x + std::exp(lp[i]));
        return v;
    }
};

// Solve M y = b (dense, partial pivoting); false if singular.
bool solve(std::vector<double> M, std::vector<double> &b, int n) {
    for (int c = 0; c < n; c++) {
        int piv = c;
        for (int r = c + 1; r < n; r++)
            if (std::fabs(M[r * n + c]) > std::fabs(M[piv * n + c])) piv = r;
        if (!(std::fabs(M[piv * n + c]) > 0)) return false;
        if (piv != c) {
            for (int j = 0; j < n; j++) std::swap(M[c * n + j], M[piv * n + j]);
            std::swap(b[c], b[piv]);
        }
        for (int r = c + 1; r < n; r++) {
            const double f = M[r * n + c] / M[c * n + c];
            if (f == 0) continue;
            for (int j = c; j < n; j++) M[r * n + j] -= f * M[c * n + j];
            b[r] -= f * b[c];
        }
    }
    for (int r = n - 1; r >= 0; r--) {
        double s = b[r];
        for (int j = r + 1; j < n; j++) s -= M[r * n + j] * b[j];
        b[r] = s / M[r * n + r];
    }
    return true;
}

// Newton on e(x_k) = (-1)^k delta, k = 0..2n+1.  Unknowns: logA, lz, lp, delta.
bool newton(Rat &R, double &delta, const std::vector<double> &xs) {
    const int n = R.n, m = 2 * n + 2;
    for (int it = 0; it < 60; it++) {
        std::vector<double> J((size_t)m * m, 0.0), f(m);
        double fmax = 0;
        for (int k = 0; k < m; k++) {
            const double x = xs[k], sg = (k & 1) ? -1.0 : 1.0;
            f[k] = -(R.err(x) - sg * delta);
            fmax = std::max(fmax, std::fabs(f[k]));
            double *row = &J[(size_t)k * m];
            row[0] = 1.0;
            for (int i = 0; i < n; i++) {
                const double z = std::exp(R.lz[i]), p = std::exp(R.lp[i]);
                row[1 + i] = z / (x + z);
                row[1 + n + i] = -p / (x + p);
            }
            row[m - 1] = -sg;
        }
        if (!solve(J, f, m)) return false;
        double step = 0;
        for (int j = 0; j < m; j++) step = std::max(step, std::fabs(f[j]));
        // damp large steps in the logarithms
        const double damp = step > 1.0 ? 1.0 / step : 1.0;
        R.logA += damp * f[0];
        for (int i = 0; i < n; i++) {
            R.lz[i] += damp * f[1 + i];
            R.lp[i] += damp * f[1 + n + i];
        }
        delta += damp * f[m - 1];
        if (step < 1e-14 && fmax < 1e-15) return true;
        if (step < 1e-13) return true;
    }
    return true;
}

// The 2n+2 alternating extrema of e on [a, b] (endpoints included), from a
// log-spaced grid refined by golden-section search on every local extremum.
bool extrema(const Rat &R, double a, double b, std::vector<double> &xs) {
    const int m = 2 * R.n + 2;
    const int G = 20000;
    std::vector<double> t(G + 1), v(G + 1);
    for (int i = 0; i <= G; i++) {
        t[i] = std::log(a) + (std::log(b) - std::log(a)) * i / G;
        v[i] = R.err(std::exp(t[i]));
    }
    std::vector<double> cand, cval;
    auto refine = [&](int i) {
        // golden-section on |e| in [t[i-1], t[i+1]]
        double lo = t[std::max(i - 1, 0)], hi = t[std::min(i + 1, G)];
        const double sgn = v[i] >= 0 ? 1.0 : -1.0;
        const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
        double c = hi - gr * (hi - lo), d = lo + gr * (hi - lo);
        for (int it = 0; it < 80; it++) {
            if (sgn * R.err(std::exp(c)) > sgn * R.err(std::exp(d)))
                hi = d;
            else
                lo = c;
            c = hi - gr * (hi - lo);
            d = lo + gr * (hi - lo);
        }
        return 0.5 * (lo + hi);
    };
    cand.push_back(t[0]);
    cval.push_back(v[0]);
    for (int i = 1; i < G; i++)
        if ((v[i] >= v[i - 1] && v[i] >= v[i + 1]) || (v[i] <= v[i - 1] && v[i] <= v[i + 1])) {
            const double tt = refine(i);
            cand.push_back(tt);
            cval.push_back(R.err(std::exp(tt)));
        }
    cand.push_back(t[G]);
    cval.push_back(v[G]);
    // merge runs of equal sign keeping the largest modulus
    std::vector<double> xt, xv;
    for (size_t i = 0; i < cand.size(); i++) {
        if (!xv.empty() && (xv.back() >= 0) == (cval[i] >= 0)) {
            if (std::fabs(cval[i]) > std::fabs(xv.back())) {
                xv.back() = cval[i];
                xt.back() = cand[i];
            }
        } else {
            xt.push_back(cand[i]);
            xv.push_back(cval[i]);
        }
    }
    // keep m consecutive alternating points containing the largest |e|
    while ((int)xt.size() > m) {
        if (std::fabs(xv.front()) < std::fabs(xv.back())) {
            xt.erase(xt.begin());
            xv.erase(xv.begin());
        } else {
            xt.pop_back();
            xv.pop_back();
        }
    }
    if ((int)xt.size() != m) return false;
    xs.resize(m);
    for (int k = 0; k < m; k++) xs[k] = std::exp(xt[k]);
    return true;
}

}  // namespace
}  // namespace cstar

using namespace cstar;

extern "C" cstar_status cstar_ratapprox_quartic(int n, double ra, double rb, double *A, double *nu2, double *mu2,
                                                double *delta) {
    if (n < 1 || n > 32 || !(ra > 0) || !(rb > ra) || !std::isfinite(rb) || !A || !nu2 || !mu2 || !delta)
        return fail(CSTAR_EINVAL, "cstar_ratapprox_quartic: bad argument");
    Rat R;
    R.n = n;
    R.lz.resize(n);
    R.lp.resize(n);
    // start: poles and zeros interlaced on a logarithmic scale beyond both ends
    const double la = std::log(ra), lb = std::log(rb), w = lb - la;
    for (int i = 0; i < n; i++) {
        R.lp[i] = la - 0.1 * w + 1.2 * w * (i + 0.25) / n;
        R.lz[i] = la - 0.1 * w + 1.2 * w * (i + 0.75) / n;
    }
    R.logA = 0.0;
    {
        // least-squares constant: zero mean of e on a grid
        double s = 0;
        const int G = 400;
        for (int i = 0; i <= G; i++) s += R.err(std::exp(la + w * i / G));
        R.logA = -s / (G + 1);
    }
    const int m = 2 * n + 2;
    std::vector<double> xs(m);
    for (int k = 0; k < m; k++) xs[k] = std::exp(la + w * 0.5 * (1.0 - std::cos(M_PI * k / (m - 1))));
    double d = 0.0;
    double dmax = 0.0;
    for (int outer = 0; outer < 100; outer++) {
        Rat save = R;
        if (!newton(R, d, xs)) return fail(CSTAR_ENOCONV, "cstar_ratapprox_quartic: Newton step failed");
        if (!std::isfinite(d)) return fail(CSTAR_ENOCONV, "cstar_ratapprox_quartic: diverged");
        std::vector<double> nx;
        if (!extrema(R, ra, rb, nx)) return fail(CSTAR_ENOCONV, "cstar_ratapprox_quartic: no alternation");
        double emax = 0, emin = 1e300;
        for (double x : nx) {
            const double e = std::fabs(R.err(x));
            emax = std::max(emax, e);
            emin = std::min(emin, e);
        }
        xs = nx;
        dmax = emax;
        (void)save;
        if (emax - emin <= 1e-9 * emax) break;
    }
    // poles and zeros sorted ascending
    std::vector<double> z(n), p(n);
    for (int i = 0; i < n; i++) {
        z[i] = std::exp(R.lz[i]);
        p[i] = std::exp(R.lp[i]);
    }
    std::sort(z.begin(), z.end());
    std::sort(p.begin(), p.end());
    *A = std::exp(R.logA);
    for (int i = 0; i < n; i++) {
        nu2[i] = z[i];
        mu2[i] = p[i];
    }
    *delta = dmax;
    return CSTAR_OK;
}
