// Lowest |eigenvalues| of Q(m) = g5 D(m) on the GPU: block Chebyshev-Davidson
// iteration on A = Q^2 (Zhou & Saad, "A Chebyshev-Davidson algorithm for large
// symmetric eigenproblems", SIAM J. Matrix Anal. Appl. 29 (2007)) with
// Rayleigh-Ritz in FP64, followed by Rayleigh-Ritz with Q itself in the
// converged subspace to give signed eigenvalues and rigorous residual bounds.
//
// The spectrum of Q is doubly degenerate (paper: v and C T g5 v^* are
// orthogonal eigenvectors with the same eigenvalue), so k eigenvalues counted
// once per pair need a block of at least 2k vectors.  Each iteration:
//   Y = p_d(A) X        Chebyshev filter of degree d damping [a_cut, b_up]
//   Y <- orth(Y - X X^H Y)                       FP64, SVQB orthonormalisation
//   [X Y] Rayleigh-Ritz with A in FP64 (A applied in FP64) -> keep nb lowest
//   Rayleigh-Ritz of Q on X -> signed lambda, residuals ||Q z - lambda z||
// Plain FP64 form: the filter in FP64.  Mixed forms: the filter acts on the
// deflated block p(A) X - X p(Theta) (same span with X), driven by the FP64
// residuals, in FP32 arithmetic with BF16 (then FP32) links; its rounding is
// relative to the residuals, so the iteration converges to FP64 accuracy
// without FP64 filtering.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "blas.h"
#include "cstar_internal.h"
#include "dense_eig.h"
#include "eig.h"
#include "nn.h"

namespace cstar {

constexpr int kMaxDegree = 800;  // largest Chebyshev degree of one filter

struct Workspace {
    int nb = 0;
    int extra = 0;              // additional Y / T slots (preconditioned residuals)
    long n = 0;                 // complex entries per FP64 vector
    double2 *XY = nullptr;      // 2nb + extra vectors: X = [0,nb), Y = [nb,2nb+extra)
    double2 *AXY = nullptr;     // 2nb + extra vectors: A X, A Y
    double2 *T = nullptr;       // nb + extra vectors
    double2 *T2 = nullptr;      // nb + extra vectors
    float4 *F[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // FP32 filter blocks (nb each)
    float *coef = nullptr;              // per-vector recurrence coefficients [kMaxDegree][nb] (device)
    std::vector<float> coef_host;       // their host staging copy (alive until the copy completes)
    double2 *partial = nullptr;
    double2 *G = nullptr;       // device small matrix (up to 128 x 128)
    double2 *C = nullptr;
    int warm_nb = 0;            // > 0: X holds the Ritz block of the last converged call
    std::vector<void *> owned;
};

static void ws_free(Workspace *w) {
    if (!w) return;
    for (void *p : w->owned) (void)hipFree(p);
    delete w;
}

void workspace_release(cstar_gauge *g) {
    ws_free(g->ws);
    g->ws = nullptr;
}

static cstar_status ws_get(cstar_gauge *g, int nb, int extra, Workspace **out) {
    const long n = n_cplx(g->geo);
    if (g->ws && g->ws->nb >= nb && g->ws->extra >= extra && g->ws->n == n) {
        *out = g->ws;
        return CSTAR_OK;
    }
    workspace_release(g);
    Workspace *w = new Workspace();
    w->nb = nb;
    w->extra = extra;
    w->n = n;
    auto alloc = [&](size_t bytes, void **p) -> bool {
        if (hipMalloc(p, bytes) != hipSuccess) return false;
        w->owned.push_back(*p);
        return true;
    };
    const size_t v64 = (size_t)n * sizeof(double2), v32 = (size_t)n / 2 * sizeof(float4);
    bool ok = alloc((2 * nb + extra) * v64, (void **)&w->XY) && alloc((2 * nb + extra) * v64, (void **)&w->AXY) &&
              alloc((nb + extra) * v64, (void **)&w->T) && alloc((nb + extra) * v64, (void **)&w->T2) &&
              alloc(gram_partial_bytes(), (void **)&w->partial) && alloc(128 * 128 * sizeof(double2), (void **)&w->G) &&
              alloc(128 * 128 * sizeof(double2), (void **)&w->C);
    for (int i = 0; i < 5 && ok; i++) ok = alloc(nb * v32, (void **)&w->F[i]);
    ok = ok && alloc(sizeof(float) * kMaxDegree * nb, (void **)&w->coef);
    if (!ok) {
        (void)hipGetLastError();
        ws_free(w);
        return fail(CSTAR_ENOMEM, "eigensolver workspace allocation failed");
    }
    g->ws = w;
    *out = w;
    return CSTAR_OK;
}

namespace {

struct Ctx {
    cstar_gauge *g;
    Workspace *w;
    hipStream_t s;
    double m;
    long ap64 = 0, ap_inner = 0, nn_applies = 0;
};

// Preconditioned residuals of the nr lowest Ritz pairs into R (FP64):
//   R_j = M (A x_j - theta_j x_j),
// with the attached network M ~ A^-1 applied in FP32, or M = 1 (the residuals
// themselves).  For M close to A^-1 on the modes above the wanted ones,
// M r_j approximates the error of x_j, so these directions complement the
// Chebyshev-filtered block (a block Davidson / LOBPCG-style correction).
cstar_status precond_residuals(Ctx &c, const double2 *X, const double2 *AX, const double *theta, int nr, double2 *R,
                               bool network) {
    const long n = c.w->n;
    CSTAR_HIP(hipMemcpyAsync(R, AX, sizeof(double2) * n * nr, hipMemcpyDeviceToDevice, c.s));
    for (int j = 0; j < nr; j++)
        CSTAR_HIP(launch_lincomb64(2 * n, -theta[j], (const double *)(X + j * n), 1.0, (double *)(R + j * n), 0.0,
                                   nullptr, c.s));
    if (!network) return CSTAR_OK;
    CSTAR_HIP(launch_to_f32(c.g->geo, nr, R, c.w->F[0], c.s));
    cstar_status st = nn_apply_block(c.g, c.w->F[0], nr);
    if (st) return st;
    c.nn_applies += nr;
    CSTAR_HIP(launch_to_f64(c.g->geo, nr, c.w->F[0], R, c.s));
    return CSTAR_OK;
}

// out = ea * Q in [+ eb * y + ec * z] on nv FP64 vectors
hipError_t q64(Ctx &c, const double2 *in, double2 *out, int nv, double ea = 1.0, const double2 *y = nullptr,
               double eb = 0.0, const double2 *z = nullptr, double ec = 0.0) {
    ApplyArgs a{in, out, (long)c.w->n * (long)sizeof(double2), nv, 1, nullptr, c.m};
    a.y = y;
    a.z = z;
    a.ea = ea;
    a.eb = eb;
    a.ec = ec;
    c.ap64 += nv;
    return handle_apply(c.g, CSTAR_FP64, a);
}
hipError_t q32(Ctx &c, cstar_prec prec, const float4 *in, float4 *out, int nv, double ea = 1.0,
               const float4 *y = nullptr, double eb = 0.0, const float4 *z = nullptr, double ec = 0.0,
               const float4 *w = nullptr, const float *ew = nullptr, double shift = 0.0) {
    ApplyArgs a{in, out, (long)c.w->n / 2 * (long)sizeof(float4), nv, 1, nullptr, c.m};
    a.shift = shift;
    a.y = y;
    a.z = z;
    a.ea = ea;
    a.eb = eb;
    a.ec = ec;
    a.w = w;
    a.ew = ew;
    c.ap_inner += nv;
    return handle_apply(c.g, prec, a);
}

// host copy of a device gram matrix V^H W (nv x nw), tiled in 64 x 64 pieces
cstar_status gram(Ctx &c, const double2 *V, int nv, const double2 *W, int nw, std::vector<zd> &G) {
    G.assign((size_t)nv * nw, zd(0, 0));
    const long n = c.w->n;
    std::vector<double2> tile(64 * 64);
    for (int i0 = 0; i0 < nv; i0 += 64)
        for (int j0 = 0; j0 < nw; j0 += 64) {
            const int bi = std::min(64, nv - i0), bj = std::min(64, nw - j0);
            CSTAR_HIP(launch_gram(V + (long)i0 * n, n, bi, W + (long)j0 * n, n, bj, n, c.w->partial, c.w->G, c.s));
            CSTAR_HIP(hipMemcpyAsync(tile.data(), c.w->G, sizeof(double2) * bi * bj, hipMemcpyDeviceToHost, c.s));
            CSTAR_HIP(hipStreamSynchronize(c.s));
            for (int i = 0; i < bi; i++)
                for (int j = 0; j < bj; j++)
                    G[(size_t)(i0 + i) * nw + j0 + j] = zd(tile[i * bj + j].x, tile[i * bj + j].y);
        }
    return CSTAR_OK;
}

// O = beta O + V C with C (nv x no) host row-major
cstar_status combine(Ctx &c, const double2 *V, int nv, const std::vector<zd> &C, int no, double2 *O,
                     double beta = 0.0) {
    std::vector<double2> h((size_t)nv * no);
    for (size_t i = 0; i < h.size(); i++) h[i] = make_double2(C[i].real(), C[i].imag());
    CSTAR_HIP(hipMemcpyAsync(c.w->C, h.data(), sizeof(double2) * h.size(), hipMemcpyHostToDevice, c.s));
    CSTAR_HIP(launch_combine(V, c.w->n, nv, c.w->C, no, O, c.w->n, no, c.w->n, c.s, beta));
    CSTAR_HIP(hipStreamSynchronize(c.s));  // C staging buffer is reused by the next call
    return CSTAR_OK;
}

// Orthonormalise the nv vectors at Y in place against themselves (SVQB:
// G = Y^H Y = U S U^H, Y <- Y U S^{-1/2}, dropping directions below drop_tol).
// Returns the number of vectors kept (compacted to the front of Y).
cstar_status orthonormalise(Ctx &c, double2 *Y, int nv, double2 *tmp, int *kept) {
    std::vector<zd> G;
    cstar_status st = gram(c, Y, nv, Y, nv, G);
    if (st) return st;
    std::vector<double> d(nv);
    for (int i = 0; i < nv; i++) d[i] = std::sqrt(std::max(G[(size_t)i * nv + i].real(), 1e-300));
    std::vector<zd> Gs((size_t)nv * nv);
    for (int i = 0; i < nv; i++)
        for (int j = 0; j < nv; j++) Gs[(size_t)i * nv + j] = G[(size_t)i * nv + j] / (d[i] * d[j]);
    std::vector<double> w;
    std::vector<zd> U;
    herm_eig(nv, Gs, w, U);
    const double wmax = w.empty() ? 0.0 : w.back();
    std::vector<int> keep;
    for (int j = nv - 1; j >= 0; j--)
        if (w[j] > 1e-13 * wmax) keep.push_back(j);
    const int nk = (int)keep.size();
    std::vector<zd> Cm((size_t)nv * nk);
    for (int i = 0; i < nv; i++)
        for (int jj = 0; jj < nk; jj++) Cm[(size_t)i * nk + jj] = U[(size_t)i * nv + keep[jj]] / (d[i] * std::sqrt(w[keep[jj]]));
    st = combine(c, Y, nv, Cm, nk, tmp);
    if (st) return st;
    CSTAR_HIP(hipMemcpyAsync(Y, tmp, sizeof(double2) * c.w->n * nk, hipMemcpyDeviceToDevice, c.s));
    *kept = nk;
    return CSTAR_OK;
}

// Y <- Y - X (X^H Y)
cstar_status project_out(Ctx &c, const double2 *X, int nx, double2 *Y, int ny) {
    std::vector<zd> G;
    cstar_status st = gram(c, X, nx, Y, ny, G);
    if (st) return st;
    for (auto &v : G) v = -v;
    return combine(c, X, nx, G, ny, Y, 1.0);
}

// Rayleigh-Ritz of H = V^H A V in the basis V (nt vectors) with its overlap
// M = V^H V (the basis is orthonormal only up to rounding): with
// M = U S U^H and B = U S^{-1/2} over the well-conditioned directions, the
// Ritz pairs are eig(B^H H B) = (theta, Z) and the Ritz vectors V B Z.
// Returns theta ascending and the coefficient matrix C = B Z (nt x r).
void rr_generalised(int nt, const std::vector<zd> &H, const std::vector<zd> &M, std::vector<double> &theta,
                    std::vector<zd> &C, int *rank) {
    std::vector<double> sg;
    std::vector<zd> U;
    herm_eig(nt, M, sg, U);
    const double smax = sg.empty() ? 0.0 : sg.back();
    std::vector<int> keep;
    for (int j = nt - 1; j >= 0; j--)
        if (sg[j] > 1e-12 * smax) keep.push_back(j);
    const int r = (int)keep.size();
    std::vector<zd> B((size_t)nt * r);
    for (int i = 0; i < nt; i++)
        for (int jj = 0; jj < r; jj++) B[(size_t)i * r + jj] = U[(size_t)i * nt + keep[jj]] / std::sqrt(sg[keep[jj]]);
    // Hr = B^H H B
    std::vector<zd> HB((size_t)nt * r, zd(0, 0)), Hr((size_t)r * r, zd(0, 0));
    for (int i = 0; i < nt; i++)
        for (int l = 0; l < nt; l++) {
            const zd h = H[(size_t)i * nt + l];
            if (h == zd(0, 0)) continue;
            for (int jj = 0; jj < r; jj++) HB[(size_t)i * r + jj] += h * B[(size_t)l * r + jj];
        }
    for (int a = 0; a < r; a++)
        for (int i = 0; i < nt; i++) {
            const zd b = std::conj(B[(size_t)i * r + a]);
            for (int jj = 0; jj < r; jj++) Hr[(size_t)a * r + jj] += b * HB[(size_t)i * r + jj];
        }
    std::vector<zd> Z;
    herm_eig(r, Hr, theta, Z);
    C.assign((size_t)nt * r, zd(0, 0));
    for (int i = 0; i < nt; i++)
        for (int l = 0; l < r; l++) {
            const zd b = B[(size_t)i * r + l];
            for (int jj = 0; jj < r; jj++) C[(size_t)i * r + jj] += b * Z[(size_t)l * r + jj];
        }
    *rank = r;
}

// Chebyshev filter Y = T_d(x(A)) X / T_d(x(a0)), x(t) = (t - cen)/e, A = Q^2.
// Three-term recurrence with the normalisation sigma_j = T_{j-1}(x0)/T_j(x0):
//   Y_1 = sigma_1/e (A - cen) X,  Y_{j+1} = 2 sigma_{j+1}/e (A - cen) Y_j - sigma_j sigma_{j+1} Y_{j-1},
//   sigma_1 = 1/x0, sigma_{j+1} = 1/(2 x0 - sigma_j).
// Each step is two Q applies; the second forms the three-term update in its
// epilogue.  FP64 buffers: three rotating blocks (Yout, B1, B2) and BQ for
// Q Y_j; X is read only.
cstar_status filter64(Ctx &c, const double2 *X, int nv, double2 *Yout, double a0, double acut, double bup, int deg,
                      double2 *B1, double2 *B2, double2 *BQ) {
    const double e = 0.5 * (bup - acut), cen = 0.5 * (bup + acut);
    const double x0 = (a0 - cen) / e;
    double sig = 1.0 / x0;
    double2 *buf[3] = {Yout, B1, B2};
    int icur = 0, iprev = -1;  // iprev = -1 means X
    CSTAR_HIP(q64(c, X, BQ, nv));
    CSTAR_HIP(q64(c, BQ, buf[icur], nv, sig / e, X, -cen * sig / e));
    for (int j = 1; j < deg; j++) {
        const double sig2 = 1.0 / (2.0 * x0 - sig);
        int inext = 0;
        while (inext == icur || inext == iprev) inext++;
        const double2 *prev = iprev < 0 ? X : buf[iprev];
        CSTAR_HIP(q64(c, buf[icur], BQ, nv));
        CSTAR_HIP(q64(c, BQ, buf[inext], nv, 2.0 * sig2 / e, buf[icur], -2.0 * sig2 * cen / e, prev, -sig * sig2));
        iprev = icur;
        icur = inext;
        sig = sig2;
    }
    if (icur != 0)
        CSTAR_HIP(hipMemcpyAsync(Yout, buf[icur], sizeof(double2) * c.w->n * nv, hipMemcpyDeviceToDevice, c.s));
    return CSTAR_OK;
}

// Deflated form of the filter for Ritz vectors X (X^H A X = diag(theta),
// X^H X = 1) with residuals R = A X - X diag(theta) (FP64).  It computes
//   Z = p(A) X - X p(diag(theta)),   p(t) = T_d(x(t)) / T_d(x(a0)),
// whose span with X equals that of [X, p(A) X].  With tau_j(m) the scalar
// recurrence at theta_m (tau_0 = 1, tau_1 = sigma_1 x(theta_m)), the
// normalised Z_j obeys
//   Z_1 = sigma_1/e R,
//   Z_{j+1} = 2 sigma_{j+1}/e (A - cen) Z_j - sigma_j sigma_{j+1} Z_{j-1} + 2 sigma_{j+1}/e R diag(tau_j),
// so the operator is only applied to Z, which is of the size of the
// residual: its rounding (FP32 arithmetic, FP32 or BF16 links) is relative to
// the residual and sets no floor on the attainable accuracy, unlike
// filtering X itself.  Buffers: F[0..3] rotate, F[4] holds R in FP32.
cstar_status filter_deflated(Ctx &c, cstar_prec prec, const double2 *X, const double2 *AX, const double *theta,
                             int nv, double2 *Yout, double a0, double acut, double bup, int deg, double2 *Rtmp) {
    Workspace *w = c.w;
    const long n = w->n;
    const double e = 0.5 * (bup - acut), cen = 0.5 * (bup + acut);
    const double x0 = (a0 - cen) / e;
    deg = std::max(1, std::min(deg, kMaxDegree));
    // R = A X - X diag(theta) in FP64, then FP32
    CSTAR_HIP(hipMemcpyAsync(Rtmp, AX, sizeof(double2) * n * nv, hipMemcpyDeviceToDevice, c.s));
    for (int m = 0; m < nv; m++)
        CSTAR_HIP(launch_lincomb64(2 * n, -theta[m], (const double *)(X + m * n), 1.0, (double *)(Rtmp + m * n), 0.0,
                                   nullptr, c.s));
    float4 *Rf = w->F[4];
    CSTAR_HIP(launch_to_f32(c.g->geo, nv, Rtmp, Rf, c.s));
    // scalar recurrences: sigma_j and tau_j(m); coefficients of R for steps j -> j+1
    std::vector<double> sig(deg + 1);
    sig[1] = 1.0 / x0;
    for (int j = 1; j < deg; j++) sig[j + 1] = 1.0 / (2.0 * x0 - sig[j]);
    std::vector<double> tprev(nv, 1.0), tcur(nv);
    for (int m = 0; m < nv; m++) tcur[m] = sig[1] * (theta[m] - cen) / e;
    w->coef_host.assign((size_t)deg * w->nb, 0.f);
    for (int j = 1; j < deg; j++) {
        for (int m = 0; m < nv; m++) {
            w->coef_host[(size_t)j * w->nb + m] = (float)(2.0 * sig[j + 1] / e * tcur[m]);
            const double tn = 2.0 * sig[j + 1] * (theta[m] - cen) / e * tcur[m] - sig[j] * sig[j + 1] * tprev[m];
            tprev[m] = tcur[m];
            tcur[m] = tn;
        }
    }
    CSTAR_HIP(hipMemcpyAsync(w->coef, w->coef_host.data(), sizeof(float) * w->coef_host.size(),
                             hipMemcpyHostToDevice, c.s));
    float4 *prev = w->F[0], *cur = w->F[1], *nxt = w->F[2], *tq = w->F[3];
    const size_t vb = (size_t)n / 2 * sizeof(float4) * nv;
    CSTAR_HIP(hipMemsetAsync(prev, 0, vb, c.s));  // Z_0 = 0
    CSTAR_HIP(hipMemsetAsync(cur, 0, vb, c.s));
    CSTAR_HIP(launch_lincomb32(2 * n * nv, (float)(sig[1] / e), (const float *)Rf, 0.f, (float *)cur, 0.f, nullptr,
                               c.s));
    // A - cen = (Q - s)(Q + s), s = sqrt(cen): the shifts enter the local mass
    // term, so the second apply needs no extra read of Z_j
    const double sh = std::sqrt(cen);
    for (int j = 1; j < deg; j++) {
        const double a = 2.0 * sig[j + 1] / e;
        CSTAR_HIP(q32(c, prec, cur, tq, nv, 1.0, nullptr, 0.0, nullptr, 0.0, nullptr, nullptr, sh));
        CSTAR_HIP(q32(c, prec, tq, nxt, nv, a, nullptr, 0.0, prev, -sig[j] * sig[j + 1], Rf,
                      w->coef + (size_t)j * w->nb, -sh));
        float4 *t = prev;
        prev = cur;
        cur = nxt;
        nxt = t;
    }
    CSTAR_HIP(launch_to_f64(c.g->geo, nv, cur, Yout, c.s));
    CSTAR_HIP(hipStreamSynchronize(c.s));  // the coefficient staging copy must finish before it is reused
    return CSTAR_OK;
}

}  // namespace

cstar_status eig_lowest(cstar_gauge *g, double m0, int k, const cstar_eig_opts *opts_in, double *evals, double *resid,
                        void *evecs, cstar_eig_stats *stats) {
    const auto t_start = std::chrono::steady_clock::now();
    cstar_eig_opts o{};
    o.inner = CSTAR_FP32_BF16LINKS;
    o.tol = 1e-10;
    o.max_iter = 200;
    if (opts_in) o = *opts_in;
    if (k < 1 || k > 30) return fail(CSTAR_EINVAL, "q_lowest_eigs: k must be in [1, 30]");
    if (!(o.tol > 0) || o.max_iter < 1) return fail(CSTAR_EINVAL, "q_lowest_eigs: bad tol/max_iter");
    // guard vectors: the low spectrum of smooth fields comes in near-degenerate
    // multiplets; the block must hold a whole multiplet beyond the wanted ones
    int nb = o.block > 0 ? o.block : 2 * k + std::max(8, k);
    nb = std::max(nb, 2 * k);
    if (nb > 64) return fail(CSTAR_EINVAL, "q_lowest_eigs: block must be <= 64");
    int deg = o.degree > 0 ? o.degree : 24;
    const int deg_max = std::max(deg, 800);
    const bool use_nn = o.use_nn == 1 && g->nn;
    const bool use_res = o.use_nn == 2;  // the residuals themselves, no network
    const int nr = (use_nn || use_res) ? std::min(2 * k, nb) : 0;  // (preconditioned) residuals per iteration
    if (nr > 0 && 2 * nb + nr > 128) return fail(CSTAR_EINVAL, "q_lowest_eigs: block too large for use_nn");
    Workspace *w = nullptr;
    cstar_status st = ws_get(g, nb, nr, &w);
    if (st) return st;
    Ctx c{g, w, g->stream, m0};
    const long n = w->n;
    double2 *X = w->XY, *Y = w->XY + (long)nb * n;
    double2 *AX = w->AXY, *AY = w->AXY + (long)nb * n;

    // rigorous upper bound of A = Q^2: ||D|| <= |4+m| + 4 + max_x ||SW(x)||
    const double qb = std::fabs(4.0 + m0) + 4.0 + std::max(0.0, g->clover_norm_max);
    const double bup = qb * qb * 1.0001;

    // start block: the previous call's Ritz block on this handle (the flow is
    // followed in small mass steps, so the low modes change little), else Gaussian
    const bool warm = o.warm_start && w->warm_nb == nb;
    if (!warm) CSTAR_HIP(launch_gauss(X, n * nb, o.seed ? o.seed : 0x5eedull, c.s));
    w->warm_nb = 0;
    int kept = 0;
    st = orthonormalise(c, X, nb, w->T, &kept);
    if (st) return st;
    if (kept < nb) return fail(CSTAR_EDEVICE, "start block lost rank");
    CSTAR_HIP(q64(c, X, w->T, nb));
    CSTAR_HIP(q64(c, w->T, AX, nb));

    std::vector<double> theta(nb, 0.0);
    double acut = bup * 0.25, a0 = 0.0;
    bool have_ritz = false;
    cstar_prec inner = o.inner;
    const char *venv = getenv("CSTAR_VERBOSE");
    const bool verbose = venv && venv[0] == '1';
    bool fp64_filter = (inner == CSTAR_FP64);
    bool refine = false;  // wanted pairs resolved: filter the leading nq vectors only
    double last_rabs = 1e300;
    int stall = 0;
    int nq = nb;  // size of the Q-reduced leading subspace (set after each RR)
    std::vector<double> lam_out(k), res_out(k);
    bool converged = false;
    int it = 0;
    for (it = 0; it < o.max_iter; it++) {
        int ny = 0;
        if (have_ritz) {
            // ---- filter.  Plain FP64 form: p(A) X in FP64.  Mixed forms: the
            // deflated filter in FP32 arithmetic (BF16, then FP32 links), whose
            // rounding is relative to the residual.  The whole block is
            // filtered until the wanted pairs are resolved, then only the
            // leading nq vectors (the guard vectors beyond the Q-reduced
            // subspace only bound the cut).
            const int nf = refine ? nq : nb;
            if (fp64_filter) {
                st = filter64(c, X, nf, Y, a0, acut, bup, deg, w->T, w->T2, AY);
            } else {
                st = filter_deflated(c, inner, X, AX, theta.data(), nf, Y, a0, acut, bup, deg, w->T2);
            }
            if (st) return st;
            // ---- learned preconditioner: append M r_j for the 2k wanted Ritz pairs
            int nin = nf;
            if (nr > 0) {
                st = precond_residuals(c, X, AX, theta.data(), nr, Y + (long)nf * n, use_nn);
                if (st) return st;
                nin = nf + nr;
            }
            // ---- orthogonalise against X twice, then orthonormalise within
            for (int r = 0; r < 2; r++) {
                st = project_out(c, X, nb, Y, nin);
                if (st) return st;
            }
            st = orthonormalise(c, Y, nin, w->T, &ny);
            if (st) return st;
            if (ny > 0) {
                CSTAR_HIP(q64(c, Y, w->T, ny));
                CSTAR_HIP(q64(c, w->T, AY, ny));
            }
        }
        // ---- Rayleigh-Ritz with A on [X Y], generalised (overlap computed).
        // After the first iteration X is the previous M-orthonormal Ritz block:
        // X^H A X = diag(theta) and X^H X = 1 are known; the Y columns are
        // formed with one pass over [X Y] for each of A Y and Y.
        const int nt = nb + ny;
        std::vector<zd> H((size_t)nt * nt, zd(0, 0)), Mo((size_t)nt * nt, zd(0, 0));
        if (!have_ritz) {
            st = gram(c, X, nb, AX, nb, H);
            if (st) return st;
            st = gram(c, X, nb, X, nb, Mo);
            if (st) return st;
        } else {
            for (int i = 0; i < nb; i++) {
                H[(size_t)i * nt + i] = theta[i];
                Mo[(size_t)i * nt + i] = 1.0;
            }
            if (ny > 0) {
                std::vector<zd> GA, GM;
                st = gram(c, w->XY, nt, AY, ny, GA);
                if (st) return st;
                st = gram(c, w->XY, nt, Y, ny, GM);
                if (st) return st;
                for (int i = 0; i < nt; i++)
                    for (int j = 0; j < ny; j++) {
                        H[(size_t)i * nt + nb + j] = GA[(size_t)i * ny + j];
                        Mo[(size_t)i * nt + nb + j] = GM[(size_t)i * ny + j];
                        if (i < nb) {
                            H[(size_t)(nb + j) * nt + i] = std::conj(GA[(size_t)i * ny + j]);
                            Mo[(size_t)(nb + j) * nt + i] = std::conj(GM[(size_t)i * ny + j]);
                        }
                    }
            }
        }
        std::vector<double> th;
        std::vector<zd> S;
        int rank = 0;
        rr_generalised(nt, H, Mo, th, S, &rank);
        if (rank < nb) return fail(CSTAR_EDEVICE, "q_lowest_eigs: search basis lost rank");
        std::vector<zd> Sk((size_t)nt * nb);
        for (int i = 0; i < nt; i++)
            for (int j = 0; j < nb; j++) Sk[(size_t)i * nb + j] = S[(size_t)i * rank + j];
        st = combine(c, w->XY, nt, Sk, nb, w->T);
        if (st) return st;
        st = combine(c, w->AXY, nt, Sk, nb, w->T2);
        if (st) return st;
        CSTAR_HIP(hipMemcpyAsync(X, w->T, sizeof(double2) * n * nb, hipMemcpyDeviceToDevice, c.s));
        CSTAR_HIP(hipMemcpyAsync(AX, w->T2, sizeof(double2) * n * nb, hipMemcpyDeviceToDevice, c.s));
        for (int j = 0; j < nb; j++) theta[j] = th[j];
        a0 = std::max(0.0, std::min(theta[0], theta[0] - 0.01 * (theta[nb - 1] - theta[0])));
        acut = theta[nb - 1];
        if (acut >= bup) acut = 0.5 * bup;
        have_ritz = true;

        // ---- signed Rayleigh-Ritz with Q on the leading nq Ritz vectors of A.
        // An eigenspace of A = Q^2 holds both +lambda and -lambda when both
        // occur (near-free fields have such multiplets); Q is reduced only on a
        // complete one, so the subspace ends at the largest relative gap of the
        // A-Ritz values at or beyond the 2k wanted ones.  QX in the Y slot.
        nq = nb;
        {
            double best = -1.0;
            for (int j = 2 * k; j < nb; j++) {
                const double gap = (theta[j] - theta[j - 1]) / std::max(theta[j], 1e-300);
                if (gap > best) {
                    best = gap;
                    nq = j;
                }
            }
        }
        CSTAR_HIP(q64(c, X, Y, nq));
        std::vector<zd> HQ;
        st = gram(c, X, nq, Y, nq, HQ);
        if (st) return st;
        std::vector<zd> MX((size_t)nq * nq, zd(0, 0));
        for (int i = 0; i < nq; i++) MX[(size_t)i * nq + i] = 1.0;
        std::vector<double> lq;
        std::vector<zd> SQfull;
        int rq = 0;
        rr_generalised(nq, HQ, MX, lq, SQfull, &rq);
        if (rq < nq) return fail(CSTAR_EDEVICE, "q_lowest_eigs: Ritz block lost rank");
        std::vector<zd> &SQ = SQfull;
        // R = Q X S - X S diag(lq) = [X, QX] [-S L; S]  (QX at column nb of XY)
        std::vector<zd> RC((size_t)(nb + nq) * nq, zd(0, 0));
        for (int i = 0; i < nq; i++)
            for (int j = 0; j < nq; j++) {
                RC[(size_t)i * nq + j] = -SQ[(size_t)i * nq + j] * lq[j];
                RC[(size_t)(nb + i) * nq + j] = SQ[(size_t)i * nq + j];
            }
        st = combine(c, w->XY, nb + nq, RC, nq, w->T);
        if (st) return st;
        std::vector<zd> RR;
        st = gram(c, w->T, nq, w->T, nq, RR);
        if (st) return st;
        std::vector<double> rn(nq);
        for (int j = 0; j < nq; j++) rn[j] = std::sqrt(std::max(0.0, RR[(size_t)j * nq + j].real()));
        // Kramers pairing: walk the signed Ritz values upwards and pair neighbours
        // that agree within their residuals; then order pairs by |lambda|.
        std::vector<int> ord(nq);
        for (int j = 0; j < nq; j++) ord[j] = j;
        std::sort(ord.begin(), ord.end(), [&](int a, int b) { return lq[a] < lq[b]; });
        struct Pr { double lam, err; int a; };
        std::vector<Pr> prs;
        std::vector<char> paired(nq, 0);
        const double qscale = std::sqrt(bup);
        for (int i = 0; i + 1 < nq;) {
            const int a = ord[i], b = ord[i + 1];
            const double gap = std::fabs(lq[a] - lq[b]);
            if (gap <= 2.0 * (rn[a] + rn[b]) + 1e-13 * qscale) {
                prs.push_back({0.5 * (lq[a] + lq[b]), std::max(rn[a], rn[b]) + 0.5 * gap, a});
                paired[a] = paired[b] = 1;
                i += 2;
            } else {
                i += 1;
            }
        }
        std::sort(prs.begin(), prs.end(), [](const Pr &x, const Pr &y) {
            const double fa = std::fabs(x.lam), fb = std::fabs(y.lam);
            return fa != fb ? fa < fb : x.lam < y.lam;
        });
        bool ok = (int)prs.size() >= k;
        double rmax = ok ? 0.0 : 1e300;
        // converged: residual below tol relative to |lambda| (floored at 1e-3), or
        // at the FP64 rounding level of the residual itself (~ eps * ||Q|| * sqrt(dim))
        const double noise = 256.0 * 2.2e-16 * qscale;
        for (int i = 0; i < k && i < (int)prs.size(); i++) {
            lam_out[i] = prs[i].lam;
            res_out[i] = prs[i].err;
            const double target = std::max(o.tol * std::max(std::fabs(lam_out[i]), 1e-3), noise);
            if (res_out[i] > target) ok = false;
            rmax = std::max(rmax, res_out[i] / std::max(std::fabs(lam_out[i]), 1e-3));
        }
        if (verbose)
            fprintf(stderr, "[cstar eig] m=%.6f it=%d nb=%d nq=%d ny=%d deg=%d pairs=%zu filter=%s acut=%.3e rmax=%.3e lam0=%.6e res0=%.2e\n",
                    m0, it, nb, nq, ny, deg, prs.size(), fp64_filter ? "fp64" : (inner == CSTAR_FP32 ? "fp32" : "bf16"), acut, rmax, prs.empty() ? 0.0 : prs[0].lam,
                    prs.empty() ? 0.0 : prs[0].err);
        // Completeness of the list: a signed Ritz value without a Kramers partner
        // whose error interval reaches down into the wanted range may be a low
        // mode not yet resolved (its partner still outside the subspace), so the
        // k listed pairs are not yet known to be the lowest: keep iterating.
        int unpaired_low = 0;
        if (ok) {
            const double reach = std::fabs(lam_out[k - 1]) + res_out[k - 1];
            for (int j = 0; j < nq; j++)
                if (!paired[j] && std::fabs(lq[j]) - rn[j] <= reach) unpaired_low++;
            if (unpaired_low) ok = false;
        }
        if (ok) {
            converged = true;
            if (evecs) {
                std::vector<zd> Sv((size_t)nq * k);
                for (int i = 0; i < nq; i++)
                    for (int j = 0; j < k; j++) Sv[(size_t)i * k + j] = SQ[(size_t)i * nq + prs[j].a];
                st = combine(c, X, nq, Sv, k, (double2 *)evecs);
                if (st) return st;
            }
            w->warm_nb = nb;
            it++;
            break;
        }
        // precision ladder of the mixed forms: the deflated filter has no
        // accuracy floor, so it stays with BF16 links while the wanted
        // residuals keep falling; after three iterations without progress it
        // moves to FP32 links, and after three more to the FP64 filter.
        double rabs = 0.0;
        for (int i = 0; i < k && i < (int)prs.size(); i++) rabs = std::max(rabs, prs[i].err);
        if ((int)prs.size() < k) rabs = 1e300;
        stall = (rabs > 0.8 * last_rabs) ? stall + 1 : 0;
        // last rung: the FP64 filter converges geometrically while the block
        // resolves the wanted pairs; eight iterations without a 0.8 reduction
        // mean it does not (e.g. a multiplet of A wider than the block), so the
        // call ends with ENOCONV instead of raising the degree further
        if (fp64_filter && stall >= 8) {
            CSTAR_HIP(hipStreamSynchronize(c.s));
            for (int i = 0; i < k; i++) {
                evals[i] = lam_out[i];
                if (resid) resid[i] = res_out[i];
            }
            if (stats) {
                stats->iterations = it + 1;
                stats->applies_fp64 = c.ap64;
                stats->applies_inner = c.ap_inner;
                stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
                stats->lambda_max_est = bup;
                stats->nn_applies = c.nn_applies;
                stats->nn_fallback = 0;
            }
            return fail(CSTAR_ENOCONV, "q_lowest_eigs: no progress in the FP64 filter (the block may be smaller "
                                       "than a multiplet of Q^2 at the wanted end; raise opts.block)");
        }
        if (rmax < 1e-4) refine = true;
        if (!fp64_filter && stall >= 3) {
            if (inner == CSTAR_FP32_BF16LINKS)
                inner = CSTAR_FP32;
            else
                fp64_filter = true;
            stall = 0;
        }
        // filter degree: about three e-folds of damping per iteration between the
        // slowest wanted Ritz value and the cut, ln T_d(x) ~ 2 d sqrt((a_cut - theta)/b_up)
        // (measured at 32^4: 1.5 / sqrt(gap / b_up) beats 0.7, 1, 2 and 3 times that),
        // but bounded so that the filter's gain across the wanted values stays
        // below 1e4 (inner precision) / 1e8 (FP64): a larger spread lets the
        // lowest mode swamp every column of the filtered block.
        if (o.degree <= 0) {
            if (it < 2 || (int)theta.size() < 2 * k) {
                deg = 16;
            } else {
                const double gk = std::max(acut - theta[2 * k - 1], 1e-300);
                const double g0 = std::max(acut - theta[0], gk);
                const double sk = std::sqrt(gk / bup), s0 = std::sqrt(g0 / bup);
                const double d_want = 1.5 / sk;
                const double d_range = std::log(fp64_filter ? 1e8 : 1e4) / (2.0 * (s0 - sk) + 1e-300);
                deg = (int)std::min<double>(deg_max, std::max<double>(8.0, std::min(d_want, d_range)));
            }
        }
        last_rabs = rabs;
    }
    CSTAR_HIP(hipStreamSynchronize(c.s));
    for (int i = 0; i < k; i++) {
        evals[i] = lam_out[i];
        if (resid) resid[i] = res_out[i];
    }
    if (stats) {
        stats->iterations = it;
        stats->applies_fp64 = c.ap64;
        stats->applies_inner = c.ap_inner;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        stats->lambda_max_est = bup;
        stats->nn_applies = c.nn_applies;
        stats->nn_fallback = 0;
    }
    if (!converged) return fail(CSTAR_ENOCONV, "q_lowest_eigs: max_iter reached");
    return CSTAR_OK;
}

}  // namespace cstar
