// Even-odd decomposition of the C* Wilson-clover operator (gfx950).
//
// Paper, mass-reweighting section: with the sites of the doubled lattice split
// by parity (every hop changes it),
//   D_hat = D_ee - D_eo D_oo^{-1} D_oe   on the even sites,
//   W_eo(m, m') = |det[D_oo(m') D_oo(m)^{-1}]|^{1/2},
// where D_oo keeps only the site-local term (4+m) + SW(x) of the odd sites.
// The local term commutes with g5, so it is two Hermitian 6x6 blocks per site
// (the clover blocks plus 4+m on the diagonal); the conjugate copy of a site
// carries sigma2 M^* sigma2 (see clover_add), whose inverse is sigma2 (M^-1)^*
// sigma2 and whose determinant has the same modulus.
//
//  * k_local_inv: the inverse blocks of (4+m) + SW on the odd sites in FP64
//    (Gauss-Jordan with partial pivoting), stored in the clover's Hermitian
//    packed format (6 real diagonal + 15 complex lower entries per block);
//  * k_eo_half<Fmt, ODD>: one parity of D_hat --
//      ODD:  chi(x) = D_oo^{-1}(x) [D_oe psi_e](x),  D_oe = -1/2 (hops from even sites);
//      EVEN: out(x) = (4+m+SW(x)) psi_e(x) - [D_eo chi](x), D_eo = -1/2 (hops from odd sites);
//  * k_logdet_ratio: sum over odd physical sites and both blocks of
//    log|det((4+m')+M_b)| - log|det((4+m)+M_b)| in FP64 (the two copies of a
//    site contribute equal moduli, which cancels the power 1/2), partial sums
//    per workgroup reduced in a fixed order.
#include "stencil_dev.h"

namespace cstar {

// Full 6x6 block b of the FP64 clover at pair (p, h) plus s on the diagonal.
__device__ __forceinline__ void herm6_full(const double2 *__restrict__ clov64, const Geo &g, int p, int h, int b,
                                           double s, cx<double> A[6][6]) {
    const double2 *q = clov64 + (long)(p * 36 + b * 18) * g.Vh + h;
    double re36[36];
#pragma unroll
    for (int k = 0; k < 18; k++) {
        const double2 w = q[(long)k * g.Vh];
        re36[2 * k] = w.x;
        re36[2 * k + 1] = w.y;
    }
#pragma unroll
    for (int i = 0; i < 6; i++) A[i][i] = {re36[i] + s, 0.0};
#pragma unroll
    for (int i = 1; i < 6; i++)
#pragma unroll
        for (int j = 0; j < i; j++) {
            const int k = i * (i - 1) / 2 + j;
            A[i][j] = {re36[6 + 2 * k], re36[7 + 2 * k]};
            A[j][i] = {re36[6 + 2 * k], -re36[7 + 2 * k]};
        }
}

__device__ __forceinline__ double cabs2(cx<double> a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ cx<double> cinv(cx<double> a) {
    const double n = 1.0 / cabs2(a);
    return {a.re * n, -a.im * n};
}

// Gauss-Jordan elimination with partial pivoting on [A | X], X = 1 on entry:
// A^{-1} in X.  Returns log|det A| (sum of log|pivot|).
__device__ double gj_inverse6(cx<double> A[6][6], cx<double> X[6][6]) {
    double logdet = 0.0;
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 6; j++) X[i][j] = {i == j ? 1.0 : 0.0, 0.0};
    for (int c = 0; c < 6; c++) {
        int piv = c;
        double best = cabs2(A[c][c]);
        for (int r = c + 1; r < 6; r++) {
            const double v = cabs2(A[r][c]);
            if (v > best) {
                best = v;
                piv = r;
            }
        }
        if (piv != c)
            for (int j = 0; j < 6; j++) {
                cx<double> t = A[c][j];
                A[c][j] = A[piv][j];
                A[piv][j] = t;
                t = X[c][j];
                X[c][j] = X[piv][j];
                X[piv][j] = t;
            }
        logdet += 0.5 * log(best);
        const cx<double> ip = cinv(A[c][c]);
        for (int j = 0; j < 6; j++) {
            A[c][j] = A[c][j] * ip;
            X[c][j] = X[c][j] * ip;
        }
        for (int r = 0; r < 6; r++) {
            if (r == c) continue;
            const cx<double> f = A[r][c];
            for (int j = 0; j < 6; j++) {
                A[r][j] = A[r][j] - f * A[c][j];
                X[r][j] = X[r][j] - f * X[c][j];
            }
        }
    }
    return logdet;
}

// log|det A| by elimination with partial pivoting (A is overwritten).
__device__ double logabsdet6(cx<double> A[6][6]) {
    double logdet = 0.0;
    for (int c = 0; c < 6; c++) {
        int piv = c;
        double best = cabs2(A[c][c]);
        for (int r = c + 1; r < 6; r++) {
            const double v = cabs2(A[r][c]);
            if (v > best) {
                best = v;
                piv = r;
            }
        }
        if (piv != c)
            for (int j = 0; j < 6; j++) {
                const cx<double> t = A[c][j];
                A[c][j] = A[piv][j];
                A[piv][j] = t;
            }
        logdet += 0.5 * log(best);
        const cx<double> ip = cinv(A[c][c]);
        for (int r = c + 1; r < 6; r++) {
            const cx<double> f = A[r][c] * ip;
            for (int j = c; j < 6; j++) A[r][j] = A[r][j] - f * A[c][j];
        }
    }
    return logdet;
}

// Inverse blocks of (4+m) + SW on the odd pairs (parity 1): inv64 double2 [36][Vh]
// (block b at b*18, packed as the clover), inv32 float4 [18][Vh] (nullable).
__global__ void k_local_inv(Geo g, const double2 *__restrict__ clov64, double m, double2 *__restrict__ inv64,
                            float4 *__restrict__ inv32) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 2 * g.Vh) return;
    const int b = gid / g.Vh;
    const int h = gid - b * g.Vh;
    cx<double> A[6][6], X[6][6];
    herm6_full(clov64, g, 1, h, b, 4.0 + m, A);
    (void)gj_inverse6(A, X);
    double re36[36];
    // the inverse of a Hermitian matrix is Hermitian: real diagonal, lower part
    for (int i = 0; i < 6; i++) re36[i] = X[i][i].re;
    for (int i = 1; i < 6; i++)
        for (int j = 0; j < i; j++) {
            const int k = i * (i - 1) / 2 + j;
            re36[6 + 2 * k] = 0.5 * (X[i][j].re + X[j][i].re);
            re36[7 + 2 * k] = 0.5 * (X[i][j].im - X[j][i].im);
        }
    double2 *o = inv64 + (long)(b * 18) * g.Vh + h;
    for (int k = 0; k < 18; k++) o[(long)k * g.Vh] = make_double2(re36[2 * k], re36[2 * k + 1]);
    if (inv32) {
        float4 *o32 = inv32 + (long)(b * 9) * g.Vh + h;
        for (int k = 0; k < 9; k++)
            o32[(long)k * g.Vh] = make_float4((float)re36[4 * k], (float)re36[4 * k + 1], (float)re36[4 * k + 2],
                                              (float)re36[4 * k + 3]);
    }
}

// The packed Hermitian blocks of the inverse, read as CloverIO reads the clover.
template <class R>
struct InvIO;
template <>
struct InvIO<double> {
    static __device__ __forceinline__ void load(const void *inv, const Geo &g, int h, int b, double dg[6],
                                                cx<double> o[15]) {
        const double2 *q = (const double2 *)inv + (long)(b * 18) * g.Vh + h;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const double2 w = q[(long)k * g.Vh];
            dg[2 * k] = w.x;
            dg[2 * k + 1] = w.y;
        }
#pragma unroll
        for (int k = 0; k < 15; k++) {
            const double2 w = q[(long)(3 + k) * g.Vh];
            o[k] = {w.x, w.y};
        }
    }
};
template <>
struct InvIO<float> {
    static __device__ __forceinline__ void load(const void *inv, const Geo &g, int h, int b, float dg[6],
                                                cx<float> o[15]) {
        const float4 *q = (const float4 *)inv + (long)(b * 9) * g.Vh + h;
        const float4 w0 = q[0], w1 = q[g.Vh];
        dg[0] = w0.x; dg[1] = w0.y; dg[2] = w0.z; dg[3] = w0.w;
        dg[4] = w1.x; dg[5] = w1.y;
        o[0] = {w1.z, w1.w};
#pragma unroll
        for (int k = 0; k < 7; k++) {
            const float4 w = q[(long)(2 + k) * g.Vh];
            o[1 + 2 * k] = {w.x, w.y};
            o[2 + 2 * k] = {w.z, w.w};
        }
    }
};

// out = M chi for a packed Hermitian block pair M of the lane's site, with the
// conjugate copy's sigma2 M^* sigma2 formed in registers (as clover_add).
template <class R>
__device__ __forceinline__ void herm_blocks_apply(const void *blk, const Geo &g, int h, int c, const cx<R> chi[12],
                                                  cx<R> out[12]) {
#pragma unroll
    for (int b = 0; b < 2; b++) {
        R dg[6];
        cx<R> o[15];
        InvIO<R>::load(blk, g, h, b, dg, o);
        cx<R> u[6], w[6];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const cx<R> c0 = chi[6 * b + a], c1 = chi[6 * b + 3 + a];
            u[a] = c ? mk(-c1.im, -c1.re) : c0;
            u[3 + a] = c ? mk(c0.im, c0.re) : c1;
        }
#pragma unroll
        for (int i = 0; i < 6; i++) {
            cx<R> acc = scale(u[i], dg[i]);
#pragma unroll
            for (int j = 0; j < 6; j++) {
                if (j < i) acc = cmac(acc, o[i * (i - 1) / 2 + j], u[j]);
                if (j > i) acc = cmac_conj(acc, o[j * (j - 1) / 2 + i], u[j]);
            }
            w[i] = acc;
        }
#pragma unroll
        for (int a = 0; a < 3; a++) {
            out[6 * b + a] = c ? mk(w[3 + a].im, w[3 + a].re) : w[a];
            out[6 * b + 3 + a] = c ? mk(-w[a].im, -w[a].re) : w[3 + a];
        }
    }
}

// One parity of D_hat for nrhs right-hand sides (stride between them in vector units).
//  ODD  (parity 1 sites): chi = D_oo^{-1} (-1/2 H psi)        psi: parity-0 block of `a`, chi -> parity-1 block of `o`
//  EVEN (parity 0 sites): out = (4+m+SW) psi + 1/2 H chi [g5]  psi: parity-0 block of `a`, chi: parity-1 block of `b`
// One right-hand side: lane = site index of the parity.  Several: item =
// (block of 256 sites, right-hand side), right-hand side fastest, and the
// grid (a multiple of 8) is dealt so that every XCD (the hardware sends
// workgroup w to XCD w mod 8) runs one contiguous range of items: the
// workgroups of a block of sites for all right-hand sides run together on
// one XCD, and the links, clover and inverse blocks of those sites are read
// from its L2 after the first.  The arithmetic of a lane is the same either
// way, so the bits are too.
template <class Fmt, bool ODD>
__global__ __launch_bounds__(256) void k_eo_half(Geo g, GaugeDev d, const typename Prec<Fmt>::V *__restrict__ a,
                                                 const typename Prec<Fmt>::V *__restrict__ b,
                                                 typename Prec<Fmt>::V *__restrict__ o, long stride_a, long stride_b,
                                                 long stride_o, int nrhs, double m, int gamma5, const void *inv) {
    using R = typename Prec<Fmt>::R;
    const long nsite = 2L * g.Vh;
    int j = 0;
    long rl;
    if (nrhs == 1) {
        rl = (long)blockIdx.x * blockDim.x + threadIdx.x;
    } else {
        const long w = blockIdx.x;
        const long item = (w & 7) * (long)(gridDim.x >> 3) + (w >> 3);
        j = (int)(item % nrhs);
        rl = (item / nrhs) * 256 + threadIdx.x;
    }
    if (rl >= nsite) return;
    const int r = (int)rl;
    const int c = r & 1;
    const int h = r >> 1;
    const int p = ODD ? 1 : 0;
    int t, x1, x2, x3;
    decode(g, p, h, t, x1, x2, x3);
    const typename Prec<Fmt>::V *src = ODD ? a + j * stride_a : b + j * stride_b;  // read at parity 1 - p
    cx<R> acc[12];
#pragma unroll
    for (int k = 0; k < 12; k++) acc[k] = {R(0), R(0)};
    hop_pair<Fmt, 0, 0>(g, d, src, p, h, c, t, x1, x2, x3, acc);
    pin(acc);
    hop_pair<Fmt, 1, 0>(g, d, src, p, h, c, t, x1, x2, x3, acc);
    pin(acc);
    hop_pair<Fmt, 2, 0>(g, d, src, p, h, c, t, x1, x2, x3, acc);
    pin(acc);
    hop_pair<Fmt, 3, 0>(g, d, src, p, h, c, t, x1, x2, x3, acc);
    pin(acc);
    cx<R> res[12];
    if constexpr (ODD) {
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = scale(acc[k], R(-0.5));
        herm_blocks_apply<R>(inv, g, h, c, acc, res);
    } else {
        cx<R> psi[12];
        SpinorIO<R>::load(a + j * stride_a, g, 0, h, c, psi);
#pragma unroll
        for (int k = 0; k < 12; k++) res[k] = {R(0), R(0)};
        clover_add<R, false>(d, g, 0, h, c, psi, res);
        const R dm = R(4.0 + m), s5 = gamma5 ? R(-1) : R(1);
#pragma unroll
        for (int k = 0; k < 12; k++) {
            cx<R> v = res[k] + scale(psi[k], dm);
            v = {fma(R(0.5), acc[k].re, v.re), fma(R(0.5), acc[k].im, v.im)};
            res[k] = k >= 6 ? scale(v, s5) : v;
        }
    }
    SpinorIO<R>::store(o + j * stride_o, g, p, h, c, res);
}

__global__ void k_logdet_ratio(Geo g, const double2 *__restrict__ clov64, double m, double mp,
                               double *__restrict__ partial) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (gid < 2 * g.Vh) {
        const int b = gid / g.Vh;
        const int h = gid - b * g.Vh;
        cx<double> A[6][6];
        herm6_full(clov64, g, 1, h, b, 4.0 + mp, A);
        const double lp = logabsdet6(A);
        herm6_full(clov64, g, 1, h, b, 4.0 + m, A);
        v = lp - logabsdet6(A);
    }
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// y += a (g5)^k x on one FP64 even vector ([12][Vh][2] double2: component c, spin c/3)
__global__ void k_even_axpy(Geo g, double are, double aim, int g5, const double2 *__restrict__ x,
                            double2 *__restrict__ y) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long n = 24L * g.Vh;
    if (e >= n) return;
    const int comp = (int)(e / (2L * g.Vh));
    const double s = (g5 && comp >= 6) ? -1.0 : 1.0;
    const double2 v = x[e];
    double2 w = y[e];
    w.x += s * (are * v.x - aim * v.y);
    w.y += s * (are * v.y + aim * v.x);
    y[e] = w;
}

hipError_t launch_even_axpy(const Geo &g, double are, double aim, int g5, const void *x, void *y, hipStream_t s) {
    const long n = 24L * g.Vh;
    hipLaunchKernelGGL(k_even_axpy, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, are, aim, g5,
                       (const double2 *)x, (double2 *)y);
    return hipGetLastError();
}

int eo_pairs_blocks(const Geo &g) { return (2 * g.Vh + 255) / 256; }

hipError_t launch_local_inv(const Geo &g, const GaugeDev &d, double m, double2 *inv64, float4 *inv32, hipStream_t s) {
    hipLaunchKernelGGL(k_local_inv, dim3(eo_pairs_blocks(g)), dim3(256), 0, s, g, (const double2 *)d.clov64, m, inv64,
                       inv32);
    return hipGetLastError();
}

hipError_t launch_logdet_ratio(const Geo &g, const GaugeDev &d, double m, double mp, double *partial, hipStream_t s) {
    hipLaunchKernelGGL(k_logdet_ratio, dim3(eo_pairs_blocks(g)), dim3(256), 0, s, g, (const double2 *)d.clov64, m, mp,
                       partial);
    return hipGetLastError();
}

template <class Fmt>
static void eo_launch(const Geo &g, const GaugeDev &d, const EoArgs &e, hipStream_t s) {
    using V = typename Prec<Fmt>::V;
    // workgroups per right-hand side; several right-hand sides: a multiple of 8 (k_eo_half deals them by XCD)
    const long per = (2L * g.Vh + 255) / 256;
    const long nwg = e.nrhs == 1 ? per : (per * e.nrhs + 7) / 8 * 8;
    const dim3 grd((unsigned)nwg), blk(256);
    const long sv = (long)sizeof(V);
    // odd half: chi (parity-1 block of tmp) from psi (parity-0 block of in)
    hipLaunchKernelGGL((k_eo_half<Fmt, true>), grd, blk, 0, s, g, d, (const V *)e.in, (const V *)nullptr,
                       (V *)e.tmp, e.stride_in / sv, 0L, e.stride_tmp / sv, e.nrhs, e.m, 0, e.inv);
    // even half: out from psi and chi
    hipLaunchKernelGGL((k_eo_half<Fmt, false>), grd, blk, 0, s, g, d, (const V *)e.in, (const V *)e.tmp,
                       (V *)e.out, e.stride_in / sv, e.stride_tmp / sv, e.stride_out / sv, e.nrhs, e.m, e.gamma5,
                       e.inv);
}

hipError_t launch_eo_apply(const Geo &g, const GaugeDev &d, cstar_prec prec, const EoArgs &e, hipStream_t s) {
    if (prec == CSTAR_FP64)
        eo_launch<FmtF64>(g, d, e, s);
    else if (prec == CSTAR_FP32)
        eo_launch<FmtF32>(g, d, e, s);
    else
        eo_launch<FmtBF16>(g, d, e, s);
    return hipGetLastError();
}

}  // namespace cstar
