// Step A of the sign algorithm upward from the target mass (paper,
// sign-of-the-Pfaffian section, the step-A list and the closing remark that
// only lambda_bar is needed there, by the power method with Chebyshev
// acceleration on Q^-2).
//
// From the target m^(0): lambda_bar(m^(n)) and its error bound; the
// exclusion interval of m^(n) has radius r_n = lambda_bar - error (no
// eigenvalue of Q reaches zero within it, Feynman-Hellmann); m^(n+1) =
// m^(n) + c r_n.  The walk ends
//   * above m_max (no crossing possible there): the whole range from the
//     target to m_max is covered by exclusion intervals, so every path point
//     has sign +1;
//   * when lambda_bar decreases, or two consecutive intervals fail to
//     overlap, or r_n is not positive: the range [target, m^(n-1)] is
//     covered (no crossing in it), and the sign there is that of m^(n-1),
//     which the block-solver driver (step B: certified crossing counts from
//     m_max down) decides together with the path points above m^(n-1).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "cstar_internal.h"

namespace cstar {

cstar_status sign_driver(cstar_eig_provider prov, void *ctx, const double *m_path, int n, int k, double c,
                         double m_max, int *sign_out, cstar_sign_report *report);

cstar_status sign_driver_stepa(cstar_lbar_provider lbar, cstar_eig_provider prov, void *ctx, const double *m_path,
                               int n, int k, double c, double m_max, int *sign_out, cstar_sign_report *report) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!lbar || !prov || !m_path || !sign_out || n < 1 || k < 1)
        return fail(CSTAR_EINVAL, "pfaffian_sign (step A): bad arguments");
    if (!(c > 0.0 && c <= 2.0)) return fail(CSTAR_EINVAL, "pfaffian_sign (step A): c must be in (0, 2]");
    if (!std::isfinite(m_max)) return fail(CSTAR_EINVAL, "pfaffian_sign (step A): m_max not finite");
    std::vector<double> path(m_path, m_path + n);
    for (double m : path)
        if (!std::isfinite(m)) return fail(CSTAR_EINVAL, "pfaffian_sign (step A): mass not finite");
    const double target = *std::min_element(path.begin(), path.end());
    std::vector<double> ms, lbs;
    auto finish_report = [&](cstar_sign_report *rep, int n_cross) {
        if (!rep) return;
        rep->n_points = std::min((int)ms.size(), 512);
        for (int i = 0; i < rep->n_points; i++) {
            rep->m[i] = ms[i];
            rep->lambda_bar[i] = lbs[i];
        }
        rep->n_crossings = n_cross;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    };
    if (target >= m_max) {
        for (int i = 0; i < n; i++) sign_out[i] = 1;
        finish_report(report, 0);
        return CSTAR_OK;
    }
    double m = target, prev_m = 0, prev_lb = 0, prev_r = 0;
    bool have_prev = false;
    double handover = 0;
    bool covered_all = false;
    for (int step = 0;; step++) {
        if (m >= m_max) {
            covered_all = true;
            break;
        }
        if ((int)ms.size() >= 512) return fail(CSTAR_ENOCONV, "pfaffian_sign (step A): too many mass points");
        double lb = 0, err = 0;
        if (lbar(ctx, m, &lb, &err) != 0) return fail(CSTAR_ENOCONV, "pfaffian_sign (step A): lambda_bar failed");
        ms.push_back(m);
        lbs.push_back(lb);
        const double r = std::max(0.0, lb - err);
        if (have_prev && (lb < prev_lb || !(prev_r + r > m - prev_m))) {
            handover = prev_m;
            break;
        }
        if (!(r > 0.0)) {
            handover = m;
            break;
        }
        prev_m = m;
        prev_lb = lb;
        prev_r = r;
        have_prev = true;
        m = m + c * r;
    }
    if (covered_all) {
        for (int i = 0; i < n; i++) sign_out[i] = 1;
        finish_report(report, 0);
        return CSTAR_OK;
    }
    // step B on [handover, m_max]: the hand-over mass and the path points above it
    std::vector<double> p2{handover};
    std::vector<int> idx2{-1};
    for (int i = 0; i < n; i++)
        if (path[i] > handover) {
            p2.push_back(path[i]);
            idx2.push_back(i);
        }
    std::vector<int> s2(p2.size(), 0);
    cstar_sign_report r2{};
    cstar_status st = sign_driver(prov, ctx, p2.data(), (int)p2.size(), k, c, m_max, s2.data(), &r2);
    if (st != CSTAR_OK && st != CSTAR_EAMBIG) return st;
    for (int i = 0; i < n; i++) sign_out[i] = s2[0];  // points in the covered range below the hand-over
    for (size_t j = 1; j < p2.size(); j++) sign_out[idx2[j]] = s2[j];
    for (int i = 0; i < r2.n_points; i++) {
        ms.push_back(r2.m[i]);
        lbs.push_back(r2.lambda_bar[i]);
    }
    finish_report(report, r2.n_crossings);
    if (st == CSTAR_EAMBIG) return fail(CSTAR_EAMBIG, "pfaffian_sign: an eigenvalue is within its error bound of zero");
    return CSTAR_OK;
}

}  // namespace cstar
