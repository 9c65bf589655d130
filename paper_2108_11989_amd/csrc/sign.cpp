// Sign of the Pfaffian from the eigenvalue flow of Q(m) (host logic).
//
// Paper, sign-of-the-Pfaffian section: pf[CTD] = prod_n lambda_n (one
// eigenvalue of Q = g5 D per Kramers pair), positive at very large mass, so
// W_sgn(m) = (-1)^(number of zero crossings of the flow between m and a mass
// above which no crossing can occur).  Since Q'(m) = g5, every eigenvalue
// moves with |lambda_n'(m)| <= 1 (Feynman-Hellmann), hence
//   (exclusion) no crossing in (m - lambda_bar(m), m + lambda_bar(m)),
// which is what step A uses: m <- m -+ c lambda_bar(m), c slightly below 2.
//
// Order: m_max is solved first, then step A walks down to the lowest path
// point; then the segments between solved masses are certified:
// A segment [a,b] of solved masses is certified
//   (i)  crossing-free when the exclusion intervals of a and b cover it:
//        r(a) + r(b) > b - a with r = min_j (|lambda_j| - err_j), a rigorous
//        lower bound of lambda_bar;
//   (ii) otherwise by counting: choose a level g < 0 that no eigenvalue can pass
//        on [a,b] -- every computed eigenvalue at a and b lies farther than
//        (b-a) + err from g, and |g| + (b-a) + err is inside the radius where
//        the computed lists are complete -- then the number of zero crossings
//        has the parity of  #{g < lambda(b) < 0} - #{g < lambda(a) < 0};
//   (iii) otherwise a new mass is solved inside the segment (the step-A point
//        a + c lambda_bar(a), or the midpoint) and both halves are certified.
// A path point that is not solved lies in a segment certified by (i), so it
// has the parity of the segment's upper end; one in a segment certified only
// by (ii) is solved, which splits that segment.  Above m_max (a mass beyond
// which D has no zero mode) the count of negative eigenvalues is that of the
// large-mass limit, which is even.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "cstar_internal.h"

namespace cstar {

namespace {
struct Point {
    double m = 0;
    std::vector<double> ev, err;
    double lb = 0, lb_err = 0;  // lambda_bar and its error bound
    double excl = 0;            // rigorous lower bound of lambda_bar: min_j (|lambda_j| - err_j), >= 0
    double R = 0;               // completeness radius of the list
    double emax = 0;            // largest error bound
    bool amb = false;           // an eigenvalue within its error of zero
};

bool solve_point(cstar_eig_provider prov, void *ctx, double m, int k, Point &p) {
    p.m = m;
    p.ev.assign(k, 0.0);
    p.err.assign(k, 0.0);
    if (prov(ctx, m, k, p.ev.data(), p.err.data()) != 0) return false;
    p.lb = 1e300;
    p.R = 1e300;
    p.emax = 0;
    p.amb = false;
    double amax = 0, eamax = 0;
    for (int i = 0; i < k; i++) {
        const double a = std::fabs(p.ev[i]);
        if (a < p.lb) {
            p.lb = a;
            p.lb_err = p.err[i];
        }
        amax = std::max(amax, a);
        eamax = std::max(eamax, p.err[i]);
        if (a <= p.err[i]) p.amb = true;
    }
    p.emax = eamax;
    p.R = amax - eamax;
    // every eigenvalue of Q(m) lies within err_j of a listed one or beyond the
    // list's reach, so no |lambda| is below min_j (|lambda_j| - err_j): the
    // exclusion interval uses that, not the error of the smallest |lambda_j|
    p.excl = 1e300;
    for (int i = 0; i < k; i++) p.excl = std::min(p.excl, std::fabs(p.ev[i]) - p.err[i]);
    p.excl = std::max(0.0, std::min(p.excl, p.R));
    return true;
}

// Returns true and the crossing parity if rule (ii) applies to [a, b].
bool count_rule(const Point &a, const Point &b, int *parity) {
    const double D = b.m - a.m;
    const double eps = std::max(a.emax, b.emax);
    const double Rmin = std::min(a.R, b.R);
    if (a.amb || b.amb || !(Rmin > D + eps)) return false;
    double best_g = 0, best_d = -1;
    for (int s = 1; s < 64; s++) {
        const double g = -Rmin * s / 64.0;
        if (-g + D + eps >= Rmin) break;
        double dmin = 1e300;
        for (const Point *p : {&a, &b})
            for (double e : p->ev) dmin = std::min(dmin, std::fabs(e - g));
        if (dmin > best_d) {
            best_d = dmin;
            best_g = g;
        }
    }
    if (!(best_d > D + eps)) return false;
    int na = 0, nb = 0;
    for (double e : a.ev)
        if (e > best_g && e < 0) na++;
    for (double e : b.ev)
        if (e > best_g && e < 0) nb++;
    *parity = ((nb - na) % 2 + 2) % 2;
    return true;
}
}  // namespace

cstar_status sign_driver(cstar_eig_provider prov, void *ctx, const double *m_path, int n, int k, double c,
                         double m_max, int *sign_out, cstar_sign_report *report) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!prov || !m_path || !sign_out || n < 1 || k < 1) return fail(CSTAR_EINVAL, "pfaffian_sign: bad arguments");
    if (!(c > 0.0 && c <= 2.0)) return fail(CSTAR_EINVAL, "pfaffian_sign: c must be in (0, 2]");
    if (!std::isfinite(m_max)) return fail(CSTAR_EINVAL, "pfaffian_sign: m_max not finite");
    std::vector<double> path(m_path, m_path + n);
    for (double m : path)
        if (!std::isfinite(m)) return fail(CSTAR_EINVAL, "pfaffian_sign: mass not finite");
    std::vector<double> uniq(path);
    std::sort(uniq.begin(), uniq.end());
    uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());

    std::map<double, Point> pts;
    std::vector<double> order;
    const int max_points = 512;
    auto solve = [&](double m) -> bool {
        Point p;
        if (!solve_point(prov, ctx, m, k, p)) return false;
        pts[m] = p;
        order.push_back(m);
        return true;
    };
    // path points at or above m_max need no solve: no eigenvalue reaches zero
    // there and the count of negative eigenvalues is the even large-mass one
    std::vector<double> need;  // path points below m_max, ascending
    for (double m : uniq)
        if (m < m_max) need.push_back(m);
    if (!solve(m_max)) return fail(CSTAR_ENOCONV, "pfaffian_sign: eigenvalue provider failed");
    // step A downwards from m_max to the lowest path point: m <- m - c lambda_bar(m)
    if (!need.empty()) {
        const double target = need.front();
        double cur = m_max;
        while (cur > target) {
            const Point &p = pts[cur];
            const double step = p.amb ? 0.0 : c * p.excl;
            double mnew = cur - step;
            // near a crossing the steps shrink geometrically: leave the rest of
            // the way to the segment certification (midpoint splits)
            if (!(step >= 0.25 * (cur - target)) || mnew <= target) mnew = target;
            if ((int)pts.size() >= max_points) return fail(CSTAR_ENOCONV, "pfaffian_sign: too many mass points");
            if (!solve(mnew)) return fail(CSTAR_ENOCONV, "pfaffian_sign: eigenvalue provider failed");
            cur = mnew;
        }
    }

    // certify segments, inserting step-A points where needed.  A segment
    // certified by exclusion (rule (i)) holds no crossing at all, so a path
    // point inside it needs no solve; a path point inside a segment certified
    // by counting (rule (ii)) is solved, which splits the segment.
    std::map<double, int> seg_cross;  // key: lower end
    std::map<double, bool> seg_excl;  // certified by exclusion
    bool ambiguous = false;
    for (;;) {
        bool inserted = false;
        for (auto it = pts.begin(); std::next(it) != pts.end(); ++it) {
            const Point &a = it->second, &b = std::next(it)->second;
            if (seg_cross.count(a.m)) continue;
            const double D = b.m - a.m;
            if (!a.amb && !b.amb && a.excl + b.excl > D) {
                seg_cross[a.m] = 0;
                seg_excl[a.m] = true;
                continue;
            }
            int par = 0;
            if (count_rule(a, b, &par)) {
                seg_cross[a.m] = par;
                seg_excl[a.m] = false;
                continue;
            }
            // split: the step-A point a + c*lambda_bar(a) when it makes real
            // progress, else the midpoint (so that a segment holding a crossing
            // shrinks until rule (ii) applies)
            double mnew = 0.5 * (a.m + b.m);
            if (!a.amb) {
                const double step = c * a.excl;
                if (step >= 0.25 * D && a.m + step < b.m) mnew = a.m + step;
            }
            if (D < 1e-12 * std::max(1.0, std::fabs(a.m))) {
                ambiguous = true;
                seg_cross[a.m] = 0;
                seg_excl[a.m] = false;
                continue;
            }
            if ((int)pts.size() >= max_points) return fail(CSTAR_ENOCONV, "pfaffian_sign: too many mass points");
            const double a_m = a.m, b_m = b.m;
            bool placed = false;
            for (int tries = 0; tries < 4 && !placed; tries++) {
                if (!solve(mnew)) return fail(CSTAR_ENOCONV, "pfaffian_sign: eigenvalue provider failed");
                const Point &pn = pts[mnew];
                if (!pn.amb) {
                    placed = true;
                    break;
                }
                // an eigenvalue sits at zero within its error here: move off it
                const double shift = 8.0 * pn.emax + 1e-9 * (b_m - a_m);
                pts.erase(mnew);
                order.pop_back();
                mnew = (mnew + shift < b_m) ? mnew + shift : mnew - shift;
                if (!(mnew > a_m && mnew < b_m)) break;
            }
            if (!placed) {
                ambiguous = true;
                seg_cross[a_m] = 0;
                seg_excl[a_m] = false;
                continue;
            }
            inserted = true;
            break;  // the map changed: rescan
        }
        if (inserted) continue;
        // every segment is certified: solve the path points that lie inside a
        // segment certified only by counting
        for (double m : need) {
            if (pts.count(m)) continue;
            auto hi = pts.upper_bound(m);
            if (hi == pts.begin() || hi == pts.end()) continue;
            const double a_m = std::prev(hi)->first;
            if (seg_excl.count(a_m) && seg_excl[a_m]) continue;
            if ((int)pts.size() >= max_points) return fail(CSTAR_ENOCONV, "pfaffian_sign: too many mass points");
            if (!solve(m)) return fail(CSTAR_ENOCONV, "pfaffian_sign: eigenvalue provider failed");
            seg_cross.erase(a_m);
            seg_excl.erase(a_m);
            inserted = true;
        }
        if (!inserted) break;
    }

    // parity of crossings above each solved point (the top point has an even
    // count); a path point that was not solved lies in a crossing-free segment
    // and has the parity of that segment's upper end
    std::map<double, int> parity_above;
    int acc = 0;
    for (auto it = pts.rbegin(); it != pts.rend(); ++it) {
        if (it != pts.rbegin()) acc = (acc + seg_cross[it->first]) & 1;
        parity_above[it->first] = acc;
    }
    int total = 0;
    for (auto &kv : seg_cross)
        if (kv.first >= uniq.front()) total += kv.second;
    cstar_status st = CSTAR_OK;
    for (int i = 0; i < n; i++) {
        if (path[i] >= m_max) {
            sign_out[i] = 1;
            continue;
        }
        auto itp = pts.find(path[i]);
        if (itp == pts.end()) {
            const double upper = pts.upper_bound(path[i])->first;
            sign_out[i] = parity_above[upper] ? -1 : 1;
            continue;
        }
        const Point &p = itp->second;
        if (p.amb || ambiguous) {
            sign_out[i] = p.amb ? 0 : (parity_above[path[i]] ? -1 : 1);
            if (p.amb) st = CSTAR_EAMBIG;
        } else {
            sign_out[i] = parity_above[path[i]] ? -1 : 1;
        }
    }
    if (ambiguous) st = CSTAR_EAMBIG;
    if (report) {
        report->n_points = std::min((int)order.size(), 512);
        for (int i = 0; i < report->n_points; i++) {
            report->m[i] = order[i];
            report->lambda_bar[i] = pts[order[i]].lb;
        }
        report->n_crossings = total;
        report->nn_applies = 0;
        report->nn_fallbacks = 0;
        report->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (st == CSTAR_EAMBIG) return fail(CSTAR_EAMBIG, "pfaffian_sign: an eigenvalue is within its error bound of zero");
    return CSTAR_OK;
}

}  // namespace cstar
