// Device-side building blocks shared by the HIP kernels of libcstar: complex
// arithmetic, the geometry of the x-doubled C* lattice in the even/odd pair
// representation, spinor and link storage formats, and the link product.
#pragma once

#include "cstar_internal.h"

namespace cstar {

template <class R>
struct cx {
    R re, im;
};
template <class R>
__device__ __forceinline__ cx<R> mk(R a, R b) { return {a, b}; }
template <class R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <class R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
// Products are written with explicit FMAs (which product is fused is fixed),
// so that every kernel rounds a site's arithmetic the same way whatever the
// compiler would otherwise contract: launch schedules give identical bits.
template <class R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
    return {fma(a.re, b.re, -(a.im * b.im)), fma(a.re, b.im, a.im * b.re)};
}
template <class R>
__device__ __forceinline__ cx<R> scale(cx<R> a, R s) { return {a.re * s, a.im * s}; }
template <class R>
__device__ __forceinline__ cx<R> conjmul(cx<R> a, cx<R> b) {  // conj(a) * b
    return {fma(a.re, b.re, a.im * b.im), fma(a.re, b.im, -(a.im * b.re))};
}
template <class R>
__device__ __forceinline__ cx<R> mul_i(cx<R> a) { return {-a.im, a.re}; }
template <class R>
__device__ __forceinline__ cx<R> mul_mi(cx<R> a) { return {a.im, -a.re}; }
template <class R>
__device__ __forceinline__ cx<R> cj(cx<R> a) { return {a.re, -a.im}; }
// fused complex multiply-accumulate: acc + a*b, acc + conj(a)*b (four FMAs each)
template <class R>
__device__ __forceinline__ cx<R> cmac(cx<R> acc, cx<R> a, cx<R> b) {
    return {fma(-a.im, b.im, fma(a.re, b.re, acc.re)), fma(a.im, b.re, fma(a.re, b.im, acc.im))};
}
template <class R>
__device__ __forceinline__ cx<R> cmac_conj(cx<R> acc, cx<R> a, cx<R> b) {
    return {fma(a.im, b.im, fma(a.re, b.re, acc.re)), fma(-a.im, b.re, fma(a.re, b.im, acc.im))};
}
// a*b - c*d
template <class R>
__device__ __forceinline__ cx<R> cmul_sub(cx<R> a, cx<R> b, cx<R> c, cx<R> d) {
    const cx<R> t = c * d;
    return cmac(cx<R>{-t.re, -t.im}, a, b);
}

// ---------------------------------------------------------------- geometry
// LOG2L > 0: L = 2^LOG2L known at compile time (shifts); 0: runtime L.
template <int LOG2L>
__device__ __forceinline__ void decode(const Geo &g, int p, int h, int &t, int &x1, int &x2, int &x3) {
    int x3h;
    if constexpr (LOG2L > 0) {
        constexpr int L = 1 << LOG2L, Lh = L / 2;
        x3h = h & (Lh - 1);
        int r = h >> (LOG2L - 1);
        x2 = r & (L - 1);
        r >>= LOG2L;
        x1 = r & (L - 1);
        t = r >> LOG2L;
    } else {
        int r = h;
        x3h = r % g.Lh;
        r /= g.Lh;
        x2 = r % g.L;
        r /= g.L;
        x1 = r % g.L;
        t = r / g.L;
    }
    x3 = 2 * x3h + ((p + t + x1 + x2) & 1);
}
template <int LOG2L>
__device__ __forceinline__ int pair_index(const Geo &g, int t, int x1, int x2, int x3) {
    if constexpr (LOG2L > 0) return ((((((t << LOG2L) + x1) << LOG2L) + x2) << LOG2L) + x3) >> 1;
    else return (((t * g.L + x1) * g.L + x2) * g.L + x3) >> 1;
}
__device__ __forceinline__ void decode(const Geo &g, int p, int h, int &t, int &x1, int &x2, int &x3) {
    decode<0>(g, p, h, t, x1, x2, x3);
}

struct Hop {
    int h;     // in-parity index of the neighbour pair (parity 1-p)
    int flip;  // 1 if the hop lands on the other copy (C* wrap)
    int tw;    // 1 if the hop wraps in time
};

template <int MU, int LOG2L>
__device__ __forceinline__ Hop hop_fwd(const Geo &g, int t, int x1, int x2, int x3) {
    const int L = LOG2L > 0 ? (1 << LOG2L) : g.L;
    int flip = 0, tw = 0;
    if (MU == 0) { t += 1; if (t == g.T) { t = 0; tw = 1; } }
    if (MU == 1) { x1 += 1; if (x1 == L) { x1 = 0; flip = 1; } }
    if (MU == 2) { x2 += 1; if (x2 == L) { x2 = 0; flip = 1; } }
    if (MU == 3) { x3 += 1; if (x3 == L) { x3 = 0; flip = 1; } }
    return {pair_index<LOG2L>(g, t, x1, x2, x3), flip, tw};
}
template <int MU, int LOG2L>
__device__ __forceinline__ Hop hop_bwd(const Geo &g, int t, int x1, int x2, int x3) {
    const int L = LOG2L > 0 ? (1 << LOG2L) : g.L;
    int flip = 0, tw = 0;
    if (MU == 0) { if (t == 0) { t = g.T; tw = 1; } t -= 1; }
    if (MU == 1) { if (x1 == 0) { x1 = L; flip = 1; } x1 -= 1; }
    if (MU == 2) { if (x2 == 0) { x2 = L; flip = 1; } x2 -= 1; }
    if (MU == 3) { if (x3 == 0) { x3 = L; flip = 1; } x3 -= 1; }
    return {pair_index<LOG2L>(g, t, x1, x2, x3), flip, tw};
}

// Streaming (non-temporal) access for data used once per launch -- the
// clover term and the output -- so that it does not evict the spinor and link
// lines that neighbouring sites read again.
typedef float ntf4 __attribute__((ext_vector_type(4)));
typedef double ntd2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float4 load_nt(const float4 *p) {
    const ntf4 v = __builtin_nontemporal_load(reinterpret_cast<const ntf4 *>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ double2 load_nt(const double2 *p) {
    const ntd2 v = __builtin_nontemporal_load(reinterpret_cast<const ntd2 *>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ void store_nt(float4 a, float4 *p) {
    const ntf4 v = {a.x, a.y, a.z, a.w};
    __builtin_nontemporal_store(v, reinterpret_cast<ntf4 *>(p));
}
__device__ __forceinline__ void store_nt(double2 a, double2 *p) {
    const ntd2 v = {a.x, a.y};
    __builtin_nontemporal_store(v, reinterpret_cast<ntd2 *>(p));
}

// ---------------------------------------------------------------- spinor storage
// load<true>: streaming loads, for operands that one lane reads once (the
// epilogue's vectors), so that they do not displace shared link and clover
// lines from L2.
// FP64: double2 [p][12][Vh][2];  FP32: float4 [p][6][Vh][2]
template <class R>
struct SpinorIO;

template <>
struct SpinorIO<double> {
    using vec = double2;
    template <bool NT = false>
    static __device__ __forceinline__ void load(const double2 *__restrict__ b, const Geo &g, int p, int h, int c,
                                                cx<double> v[12]) {
        const double2 *q = b + ((long)p * 12 * g.Vh + h) * 2 + c;
        const long st = 2L * g.Vh;
#pragma unroll
        for (int k = 0; k < 12; k++) {
            const double2 w = NT ? load_nt(&q[k * st]) : q[k * st];
            v[k] = {w.x, w.y};
        }
    }
    static __device__ __forceinline__ void store(double2 *__restrict__ b, const Geo &g, int p, int h, int c,
                                                 const cx<double> v[12]) {
        double2 *q = b + ((long)p * 12 * g.Vh + h) * 2 + c;
        const long st = 2L * g.Vh;
#pragma unroll
        for (int k = 0; k < 12; k++) store_nt(make_double2(v[k].re, v[k].im), &q[k * st]);
    }
};

template <>
struct SpinorIO<float> {
    using vec = float4;
    template <bool NT = false>
    static __device__ __forceinline__ void load(const float4 *__restrict__ b, const Geo &g, int p, int h, int c,
                                                cx<float> v[12]) {
        const float4 *q = b + ((long)p * 6 * g.Vh + h) * 2 + c;
        const long st = 2L * g.Vh;
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const float4 w = NT ? load_nt(&q[k * st]) : q[k * st];
            v[2 * k] = {w.x, w.y};
            v[2 * k + 1] = {w.z, w.w};
        }
    }
    static __device__ __forceinline__ void store(float4 *__restrict__ b, const Geo &g, int p, int h, int c,
                                                 const cx<float> v[12]) {
        float4 *q = b + ((long)p * 6 * g.Vh + h) * 2 + c;
        const long st = 2L * g.Vh;
#pragma unroll
        for (int k = 0; k < 6; k++)
            store_nt(make_float4(v[2 * k].re, v[2 * k].im, v[2 * k + 1].re, v[2 * k + 1].im), &q[k * st]);
    }
};

// ---------------------------------------------------------------- links
// A link as used by one lane: U (3x3, possibly conjugated) and a phase e^{i phi}
// that multiplies the matrix-vector product (forward) or its conjugate (adjoint).
template <class R>
struct Link {
    cx<R> u[9];
    cx<R> ph;
};

__device__ __forceinline__ float bf_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }

template <class R>
__device__ __forceinline__ void row2_from_rows(cx<R> u[9]) {
    // row 2 = conj(row0 x row1)
    u[6] = cj(cmul_sub(u[1], u[5], u[2], u[4]));
    u[7] = cj(cmul_sub(u[2], u[3], u[0], u[5]));
    u[8] = cj(cmul_sub(u[0], u[4], u[1], u[3]));
}

// The compressed formats store the SU(3) rows and the quark phase exp(i q
// theta) apart; the phase is multiplied into the nine entries once per load
// (9 complex products), so every use of the link -- up to two hops and NR
// right-hand sides -- is a plain 3x3 product.  s = -1 for the conjugate copy.
__device__ __forceinline__ void apply_phase(Link<float> &L, float2 e, float s) {
    const cx<float> ph = {e.x, s * e.y};
#pragma unroll
    for (int r = 0; r < 9; r++) L.u[r] = L.u[r] * ph;
    L.ph = {1.f, 0.f};
}

struct FmtF64 {
    using R = double;
    static __device__ __forceinline__ void load(const GaugeDev &d, const Geo &g, int p, int mu, int h, double s,
                                                Link<double> &L) {
        const double2 *b = d.link64 + (long)(p * 4 + mu) * 9 * g.Vh + h;
#pragma unroll
        for (int r = 0; r < 9; r++) {
            const double2 w = b[(long)r * g.Vh];
            L.u[r] = {w.x, s * w.y};
        }
        L.ph = {1.0, 0.0};
    }
    static constexpr bool has_phase = false;
};

struct FmtF32 {
    using R = float;
    static __device__ __forceinline__ void load(const GaugeDev &d, const Geo &g, int p, int mu, int h, float s,
                                                Link<float> &L) {
        const float4 *b = d.link32 + (long)(p * 4 + mu) * 3 * g.Vh + h;
        const float4 a0 = b[0], a1 = b[g.Vh], a2 = b[2 * (long)g.Vh];
        L.u[0] = {a0.x, s * a0.y};
        L.u[1] = {a0.z, s * a0.w};
        L.u[2] = {a1.x, s * a1.y};
        L.u[3] = {a1.z, s * a1.w};
        L.u[4] = {a2.x, s * a2.y};
        L.u[5] = {a2.z, s * a2.w};
        row2_from_rows(L.u);
        apply_phase(L, d.phase32[(long)(p * 4 + mu) * g.Vh + h], s);
    }
    static constexpr bool has_phase = false;
};

struct FmtBF16 {
    using R = float;
    static __device__ __forceinline__ void load(const GaugeDev &d, const Geo &g, int p, int mu, int h, float s,
                                                Link<float> &L) {
        const long i = (long)(p * 4 + mu) * g.Vh + h;
        const uint4 a = d.linkbf_a[i];
        const uint2 b = d.linkbf_b[i];
        L.u[0] = {bf_lo(a.x), s * bf_hi(a.x)};
        L.u[1] = {bf_lo(a.y), s * bf_hi(a.y)};
        L.u[2] = {bf_lo(a.z), s * bf_hi(a.z)};
        L.u[3] = {bf_lo(a.w), s * bf_hi(a.w)};
        L.u[4] = {bf_lo(b.x), s * bf_hi(b.x)};
        L.u[5] = {bf_lo(b.y), s * bf_hi(b.y)};
        row2_from_rows(L.u);
        apply_phase(L, d.phase32[i], s);
    }
    static constexpr bool has_phase = false;
};

// g = V h (DAG = false) or V^H h (DAG = true) for the two spin rows of a half spinor.
template <class Fmt, bool DAG, class R>
__device__ __forceinline__ void link_mul(const Link<R> &L, const cx<R> h[6], cx<R> o[6]) {
#pragma unroll
    for (int s = 0; s < 2; s++) {
#pragma unroll
        for (int i = 0; i < 3; i++) {
            cx<R> acc = DAG ? conjmul(L.u[i], h[s * 3]) : L.u[i * 3] * h[s * 3];
#pragma unroll
            for (int j = 1; j < 3; j++) {
                if (DAG)
                    acc = cmac_conj(acc, L.u[j * 3 + i], h[s * 3 + j]);
                else
                    acc = cmac(acc, L.u[i * 3 + j], h[s * 3 + j]);
            }
            if (Fmt::has_phase) acc = DAG ? conjmul(L.ph, acc) : L.ph * acc;
            o[s * 3 + i] = acc;
        }
    }
}

}  // namespace cstar
