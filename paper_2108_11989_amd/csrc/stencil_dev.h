// Stencil building blocks shared by the Dirac-apply kernels and the even-odd
// kernels: spin projection and reconstruction of the hops, the clover's
// packed Hermitian blocks, the hopping sum of one direction and the clover
// term of one lane.
#pragma once

#include "lattice_dev.h"

namespace cstar {

// Spin projection: h = P psi for (1 + SG*g_mu) (SG = -1 forward hop, +1 backward hop),
// and reconstruction of the full 4-spinor from the transported half spinor.
template <int MU, int SG, class R>
__device__ __forceinline__ void project(const cx<R> v[12], cx<R> h[6]) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const cx<R> p0 = v[a], p1 = v[3 + a], p2 = v[6 + a], p3 = v[9 + a];
        if (MU == 0) {
            h[a] = SG < 0 ? p0 + p2 : p0 - p2;
            h[3 + a] = SG < 0 ? p1 + p3 : p1 - p3;
        } else if (MU == 1) {
            h[a] = SG < 0 ? p0 + mul_i(p3) : p0 - mul_i(p3);
            h[3 + a] = SG < 0 ? p1 + mul_i(p2) : p1 - mul_i(p2);
        } else if (MU == 2) {
            h[a] = SG < 0 ? p0 + p3 : p0 - p3;
            h[3 + a] = SG < 0 ? p1 - p2 : p1 + p2;
        } else {
            h[a] = SG < 0 ? p0 + mul_i(p2) : p0 - mul_i(p2);
            h[3 + a] = SG < 0 ? p1 - mul_i(p3) : p1 + mul_i(p3);
        }
    }
}

// acc += (1 + SG g_mu)-reconstruction of the transported half spinor g
template <int MU, int SG, class R>
__device__ __forceinline__ void accumulate(cx<R> acc[12], const cx<R> g[6]) {
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const cx<R> g0 = g[a], g1 = g[3 + a];
        acc[a] = acc[a] + g0;
        acc[3 + a] = acc[3 + a] + g1;
        if (MU == 0) {
            acc[6 + a] = SG < 0 ? acc[6 + a] + g0 : acc[6 + a] - g0;
            acc[9 + a] = SG < 0 ? acc[9 + a] + g1 : acc[9 + a] - g1;
        } else if (MU == 1) {
            acc[6 + a] = acc[6 + a] + (SG < 0 ? mul_mi(g1) : mul_i(g1));
            acc[9 + a] = acc[9 + a] + (SG < 0 ? mul_mi(g0) : mul_i(g0));
        } else if (MU == 2) {
            acc[6 + a] = SG < 0 ? acc[6 + a] - g1 : acc[6 + a] + g1;
            acc[9 + a] = SG < 0 ? acc[9 + a] + g0 : acc[9 + a] - g0;
        } else {
            acc[6 + a] = acc[6 + a] + (SG < 0 ? mul_mi(g0) : mul_i(g0));
            acc[9 + a] = acc[9 + a] + (SG < 0 ? mul_i(g1) : mul_mi(g1));
        }
    }
}

// ---------------------------------------------------------------- clover storage
// Block b (b=0: spins 0,1; b=1: spins 2,3) of the Hermitian 6x6 term, index
// i = 3*spin_in_block + colour: 6 real diagonal entries, then the 15 strictly
// lower entries M[i][j] (i > j) in row order, off(i,j) = i(i-1)/2 + j.
// NT: streaming loads, for launches that read each site's clover once (one
// right-hand side); with several right-hand sides their workgroups read the
// same lines one after another and the loads keep them in L2.
template <bool NT, class T>
__device__ __forceinline__ T clover_ld(const T *p) {
    if constexpr (NT) return load_nt(p);
    else return *p;
}
template <class R>
struct CloverIO;

template <>
struct CloverIO<double> {
    template <bool NT>
    static __device__ __forceinline__ void load(const GaugeDev &d, const Geo &g, int p, int h, int b, double dg[6],
                                                cx<double> o[15]) {
        const double2 *q = d.clov64 + (long)(p * 36 + b * 18) * g.Vh + h;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const double2 w = clover_ld<NT>(&q[(long)k * g.Vh]);
            dg[2 * k] = w.x;
            dg[2 * k + 1] = w.y;
        }
#pragma unroll
        for (int k = 0; k < 15; k++) {
            const double2 w = clover_ld<NT>(&q[(long)(3 + k) * g.Vh]);
            o[k] = {w.x, w.y};
        }
    }
};
template <>
struct CloverIO<float> {
    template <bool NT>
    static __device__ __forceinline__ void load(const GaugeDev &d, const Geo &g, int p, int h, int b, float dg[6],
                                                cx<float> o[15]) {
        const float4 *q = d.clov32 + (long)(p * 18 + b * 9) * g.Vh + h;
        const float4 w0 = clover_ld<NT>(&q[0]), w1 = clover_ld<NT>(&q[g.Vh]);
        dg[0] = w0.x; dg[1] = w0.y; dg[2] = w0.z; dg[3] = w0.w;
        dg[4] = w1.x; dg[5] = w1.y;
        o[0] = {w1.z, w1.w};
#pragma unroll
        for (int k = 0; k < 7; k++) {
            const float4 w = clover_ld<NT>(&q[(long)(2 + k) * g.Vh]);
            o[1 + 2 * k] = {w.x, w.y};
            o[2 + 2 * k] = {w.z, w.w};
        }
    }
};

template <class R>
__device__ __forceinline__ void herm6_mul(const R dg[6], const cx<R> o[15], const cx<R> u[6], cx<R> w[6]) {
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
}

// ---------------------------------------------------------------- apply kernel
template <class Fmt>
struct Prec;
template <>
struct Prec<FmtF64> {
    using R = double;
    using V = double2;
};
template <>
struct Prec<FmtF32> {
    using R = float;
    using V = float4;
};
template <>
struct Prec<FmtBF16> {
    using R = float;
    using V = float4;
};

// Hopping sum of one direction (both hops), accumulated without the -1/2
// (applied once per site); the antiperiodic time sign flips the projected
// half spinor of a wrapping hop.
template <class Fmt, int MU, int LOG2L>
__device__ __forceinline__ void hop_pair(const Geo &g, const GaugeDev &d, const typename Prec<Fmt>::V *__restrict__ in,
                                         int p, int h, int c, int t, int x1, int x2, int x3,
                                         cx<typename Prec<Fmt>::R> acc[12]) {
    using R = typename Prec<Fmt>::R;
    {  // forward: (1 - g_mu) V(x,mu) psi(x+mu)
        const Hop n = hop_fwd<MU, LOG2L>(g, t, x1, x2, x3);
        Link<R> L;
        Fmt::load(d, g, p, MU, h, c ? R(-1) : R(1), L);
        cx<R> v[12], hh[6], gg[6];
        SpinorIO<R>::load(in, g, 1 - p, n.h, c ^ n.flip, v);
        project<MU, -1>(v, hh);
        if (MU == 0) {
            const R sg = (n.tw && g.time_bc < 0) ? R(-1) : R(1);
#pragma unroll
            for (int i = 0; i < 6; i++) hh[i] = scale(hh[i], sg);
        }
        link_mul<Fmt, false>(L, hh, gg);
        accumulate<MU, -1>(acc, gg);
    }
    {  // backward: (1 + g_mu) V(x-mu,mu)^H psi(x-mu)
        const Hop n = hop_bwd<MU, LOG2L>(g, t, x1, x2, x3);
        const int cn = c ^ n.flip;
        Link<R> L;
        Fmt::load(d, g, 1 - p, MU, n.h, cn ? R(-1) : R(1), L);
        cx<R> v[12], hh[6], gg[6];
        SpinorIO<R>::load(in, g, 1 - p, n.h, cn, v);
        project<MU, 1>(v, hh);
        if (MU == 0) {
            const R sg = (n.tw && g.time_bc < 0) ? R(-1) : R(1);
#pragma unroll
            for (int i = 0; i < 6; i++) hh[i] = scale(hh[i], sg);
        }
        link_mul<Fmt, true>(L, hh, gg);
        accumulate<MU, 1>(acc, gg);
    }
}

// Clover term of one lane: the physical copy uses the stored blocks M; the
// conjugate copy uses sigma2 M^* sigma2 (its field strength is conj(F)),
// evaluated as -sigma2 conj(M sigma2 chi^*) in each chirality block.
template <class R, bool NT = true>
__device__ __forceinline__ void clover_add(const GaugeDev &d, const Geo &g, int p, int h, int c, const cx<R> chi[12],
                                           cx<R> acc[12]) {
#pragma unroll
    for (int b = 0; b < 2; b++) {
        R dg[6];
        cx<R> o[15];
        CloverIO<R>::template load<NT>(d, g, p, h, b, dg, o);
        cx<R> u[6], w[6];
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const cx<R> c0 = chi[6 * b + a], c1 = chi[6 * b + 3 + a];
            u[a] = c ? mk(-c1.im, -c1.re) : c0;      // -i conj(chi1)
            u[3 + a] = c ? mk(c0.im, c0.re) : c1;    //  i conj(chi0)
        }
        herm6_mul(dg, o, u, w);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            const cx<R> r0 = c ? mk(w[3 + a].im, w[3 + a].re) : w[a];     //  i conj(w1)
            const cx<R> r1 = c ? mk(-w[a].im, -w[a].re) : w[3 + a];       // -i conj(w0)
            acc[6 * b + a] = acc[6 * b + a] + r0;
            acc[6 * b + 3 + a] = acc[6 * b + 3 + a] + r1;
        }
    }
}

// Materialise the accumulator at this point of the program: the arithmetic of
// the hops before it cannot sink below it, which bounds the live registers to
// one direction's loads instead of all sixteen hops' (the default schedule
// loads everything first and spills).
template <class R>
__device__ __forceinline__ void pin(cx<R> acc[12]) {
#pragma unroll
    for (int k = 0; k < 12; k++) asm volatile("" : "+v"(acc[k].re), "+v"(acc[k].im));
}


}  // namespace cstar
