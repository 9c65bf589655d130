// Cyclic Jacobi for complex Hermitian matrices (Rayleigh-Ritz on the host).
//
// A rotation on rows/columns (p,q) with G_pp = G_qq = c, G_pq = s e^{i phi},
// G_qp = -s e^{-i phi}, where a_pq = r e^{i phi}, annihilates a_pq of G^H A G
// when t = s/c solves t^2 + 2 tau t - 1 = 0, tau = (a_qq - a_pp) / (2 r);
// the smaller root t = sign(tau) / (|tau| + sqrt(1 + tau^2)) is taken.
#include "dense_eig.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace cstar {

void herm_eig(int n, const std::vector<zd> &Ain, std::vector<double> &w, std::vector<zd> &Vout) {
    std::vector<zd> A(Ain);
    std::vector<zd> V((size_t)n * n, zd(0.0, 0.0));
    for (int i = 0; i < n; i++) V[(size_t)i * n + i] = 1.0;
    for (int i = 0; i < n; i++)
        for (int j = i + 1; j < n; j++) {  // symmetrise
            const zd a = 0.5 * (A[(size_t)i * n + j] + std::conj(A[(size_t)j * n + i]));
            A[(size_t)i * n + j] = a;
            A[(size_t)j * n + i] = std::conj(a);
        }
    for (int i = 0; i < n; i++) A[(size_t)i * n + i] = A[(size_t)i * n + i].real();

    double scale = 0.0;
    for (size_t i = 0; i < A.size(); i++) scale = std::max(scale, std::abs(A[i]));
    if (scale == 0.0) scale = 1.0;
    for (int sweep = 0; sweep < 100; sweep++) {
        double off = 0.0;
        for (int p = 0; p < n; p++)
            for (int q = p + 1; q < n; q++) off += std::norm(A[(size_t)p * n + q]);
        if (std::sqrt(off) <= 1e-17 * scale * n) break;
        for (int p = 0; p < n - 1; p++)
            for (int q = p + 1; q < n; q++) {
                const zd apq = A[(size_t)p * n + q];
                const double r = std::abs(apq);
                if (r <= 1e-300) continue;
                const double app = A[(size_t)p * n + p].real(), aqq = A[(size_t)q * n + q].real();
                if (r < 1e-18 * (std::abs(app) + std::abs(aqq)) && sweep > 3) {
                    A[(size_t)p * n + q] = A[(size_t)q * n + p] = 0.0;
                    continue;
                }
                const zd e = apq / r;  // e^{i phi}
                const double tau = (aqq - app) / (2.0 * r);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::abs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t);
                const double s = t * c;
                const zd gpq = s * e, gqp = -s * std::conj(e);
                // A <- A G (columns p, q)
                for (int k = 0; k < n; k++) {
                    const zd akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = akp * c + akq * gqp;
                    A[(size_t)k * n + q] = akp * gpq + akq * c;
                }
                // A <- G^H A (rows p, q)
                for (int k = 0; k < n; k++) {
                    const zd apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = c * apk + std::conj(gqp) * aqk;
                    A[(size_t)q * n + k] = std::conj(gpq) * apk + c * aqk;
                }
                A[(size_t)p * n + q] = A[(size_t)q * n + p] = 0.0;
                A[(size_t)p * n + p] = A[(size_t)p * n + p].real();
                A[(size_t)q * n + q] = A[(size_t)q * n + q].real();
                for (int k = 0; k < n; k++) {
                    const zd vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = vkp * c + vkq * gqp;
                    V[(size_t)k * n + q] = vkp * gpq + vkq * c;
                }
            }
    }
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(),
              [&](int a, int b) { return A[(size_t)a * n + a].real() < A[(size_t)b * n + b].real(); });
    w.resize(n);
    Vout.assign((size_t)n * n, zd(0.0, 0.0));
    for (int j = 0; j < n; j++) {
        w[j] = A[(size_t)idx[j] * n + idx[j]].real();
        for (int i = 0; i < n; i++) Vout[(size_t)i * n + j] = V[(size_t)i * n + idx[j]];
    }
}

}  // namespace cstar
