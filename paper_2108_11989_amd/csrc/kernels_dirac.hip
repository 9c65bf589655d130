// HIP kernels of the C* Wilson-clover operator for gfx950.
//
//  * link packing: physical SU(3) x U(1) links -> FP64 quark links, FP32 / BF16
//    compressed rows with the quark phase exp(i q theta) as an FP32 (cos, sin) pair;
//  * clover: field strength from the four plaquette leaves on the x-doubled
//    lattice, SW = (i/4) sigma_{mu nu} F_{mu nu} as two Hermitian 6x6 blocks
//    (the term commutes with g5) for the physical copy of every site;
//  * apply: one thread per site of the x-doubled lattice, the two copies of a
//    physical site in adjacent lanes so that both read the same link and
//    clover words in one wave; spin projection of every hop (rank-2 (1-+g_mu)).
//
// Operator (paper, sign-of-the-Pfaffian and setup sections; chiral basis with
// g0 = [[0,-1],[-1,0]], gk = [[0,-i s_k],[i s_k,0]], g5 = diag(1,1,-1,-1)):
//   (D psi)(x) = (4+m) psi(x) + SW(x) psi(x)
//              - 1/2 sum_mu [(1-g_mu) V(x,mu) psi(x+mu) + (1+g_mu) V(x-mu,mu)^H psi(x-mu)].
// C* on the doubled lattice: the copy of x at x1+L sees conj(U), -theta; a hop
// that leaves [0,L) in x1, x2 or x3 lands on the other copy.
#include <algorithm>
#include <functional>
#include <type_traits>

#include "stencil_dev.h"

namespace cstar {

// Epilogue of a launch: out = a * ([g5] D psi) + b * y + c * z + e_j * w, with
// y, z, w spinor blocks of the output's layout and e_j a coefficient per
// right-hand side (used by the Chebyshev recurrences to form their update
// without another pass over memory).
template <class V>
struct Epi {
    const V *y, *z;     // optional operands (null: none)
    float a, b, c;      // FP32 forms
    double ad, bd, cd;  // FP64 form
    int on;
    const V *w;         // optional fourth operand (null: none)
    const void *ew;     // its coefficients: float [nrhs] (FP32 forms) or double [nrhs] (FP64)
    double shift;       // Q + shift (with g5): local mass 4+m+shift on spins 0,1 and 4+m-shift on 2,3
};

template <class R, class V>
__device__ __forceinline__ void apply_epilogue(const Geo &g, const Epi<V> &ep, int j, long joff, int p, int h, int c,
                                               cx<R> acc[12]) {
    if (!ep.on) return;
    // one operand live at a time
    const R a = sizeof(R) == 8 ? R(ep.ad) : R(ep.a);
    const R b = sizeof(R) == 8 ? R(ep.bd) : R(ep.b);
    const R cc = sizeof(R) == 8 ? R(ep.cd) : R(ep.c);
    cx<R> w[12];
    if (ep.y) {
        SpinorIO<R>::template load<true>(ep.y + joff, g, p, h, c, w);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = {fma(b, w[k].re, a * acc[k].re), fma(b, w[k].im, a * acc[k].im)};
    } else {
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = scale(acc[k], a);
    }
    if (ep.z) {
        pin(acc);
        SpinorIO<R>::template load<true>(ep.z + joff, g, p, h, c, w);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = {fma(cc, w[k].re, acc[k].re), fma(cc, w[k].im, acc[k].im)};
    }
    if (ep.w) {
        pin(acc);
        const R e = reinterpret_cast<const R *>(ep.ew)[j];
        SpinorIO<R>::template load<true>(ep.w + joff, g, p, h, c, w);
#pragma unroll
        for (int k = 0; k < 12; k++) acc[k] = {fma(e, w[k].re, acc[k].re), fma(e, w[k].im, acc[k].im)};
    }
}

// One site of the x-doubled lattice (lane = pair x copy), one right-hand side:
// out = (4+m) chi + SW chi - 1/2 (hopping sum), optionally times g5.
template <class Fmt, int LOG2L>
__device__ __forceinline__ void site_apply(const Geo &g, const GaugeDev &d, const typename Prec<Fmt>::V *__restrict__ in,
                                           typename Prec<Fmt>::V *__restrict__ out, int p, int h, int c, int t, int x1,
                                           int x2, int x3, double mass, int gamma5,
                                           const Epi<typename Prec<Fmt>::V> &ep, int j, long joff) {
    using R = typename Prec<Fmt>::R;
    cx<R> acc[12];
#pragma unroll
    for (int k = 0; k < 12; k++) acc[k] = {R(0), R(0)};
    // the pins between directions bound the live loads (and registers) to one
    // direction's two hops
    hop_pair<Fmt, 0, LOG2L>(g, d, in, p, h, c, t, x1, x2, x3, acc);
    pin(acc);
    hop_pair<Fmt, 1, LOG2L>(g, d, in, p, h, c, t, x1, x2, x3, acc);
    pin(acc);
    hop_pair<Fmt, 2, LOG2L>(g, d, in, p, h, c, t, x1, x2, x3, acc);
    pin(acc);
    hop_pair<Fmt, 3, LOG2L>(g, d, in, p, h, c, t, x1, x2, x3, acc);
    pin(acc);
    cx<R> chi[12];
    SpinorIO<R>::load(in, g, p, h, c, chi);
    cx<R> sw[12];
#pragma unroll
    for (int k = 0; k < 12; k++) sw[k] = {R(0), R(0)};
    clover_add<R>(d, g, p, h, c, chi, sw);
    const R dmu = R(4.0 + mass + ep.shift), dml = R(4.0 + mass - ep.shift);
    const R mh = R(-0.5);
    const R s5 = gamma5 ? R(-1) : R(1);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        cx<R> o = sw[k] + scale(chi[k], k < 6 ? dmu : dml);
        o = {o.re + mh * acc[k].re, o.im + mh * acc[k].im};
        if (k >= 6) o = scale(o, s5);
        acc[k] = o;
    }
    apply_epilogue<R, typename Prec<Fmt>::V>(g, ep, j, joff, p, h, c, acc);
    SpinorIO<R>::store(out, g, p, h, c, acc);
}

// Site of lane `lane` of logical tile `tile` (a tile = one workgroup of 256
// lanes = 128 pairs x 2 copies).
//  - plain order (any L): 128 consecutive pairs of the even/odd index;
//  - blocked order (L = 16, 32, 64): a tile is 16 x2-rows x 8 x3-pairs at
//    fixed (parity, t, x1); tiles run over (x1 in a block of 4, then t, then
//    the spatial region, x1-blocks fastest, then parity).  Consecutive tiles
//    walk the time direction of one compact spatial region, so the t+-1
//    neighbours -- 16K pairs apart in memory -- are fetched while still in the
//    XCD's L2, and consecutive regions share their x1 face.
template <int LOG2L>
__device__ __forceinline__ bool tile_site(const Geo &g, int tile, int lane, int &p, int &h, int &c, int &t, int &x1,
                                          int &x2, int &x3) {
    c = lane & 1;
    if constexpr (LOG2L >= 4) {
        constexpr int L = 1 << LOG2L, Lh = L / 2;
        constexpr int nx3b = Lh / 8, nx2b = L / 16, nx1b = L / 4;
        int r = tile;
        const int x1_in = r & 3;
        r >>= 2;
        t = r % g.T;
        r /= g.T;
        const int x1b = r % nx1b;
        r /= nx1b;
        const int x2b = r % nx2b;
        r /= nx2b;
        const int x3b = r % nx3b;
        p = r / nx3b;
        if (p > 1) return false;
        const int pr = lane >> 1;
        x1 = x1b * 4 + x1_in;
        x2 = x2b * 16 + (pr >> 3);
        const int x3h = x3b * 8 + (pr & 7);
        x3 = 2 * x3h + ((p + t + x1 + x2) & 1);
        h = pair_index<LOG2L>(g, t, x1, x2, x3);
        return true;
    } else {
        const int gid = tile * 256 + lane;
        if (gid >= 4 * g.Vh) return false;
        const int pair = gid >> 1;
        p = pair >= g.Vh;
        h = pair - p * g.Vh;
        decode<LOG2L>(g, p, h, t, x1, x2, x3);
        return true;
    }
}

// Workgroup w of a launch handles logical tile (w mod 8) * (nwg/8) + w/8:
// the hardware deals workgroups round-robin over the eight XCDs (w mod 8) and
// each XCD has its own L2, so every XCD gets one contiguous range of tiles.
__device__ __forceinline__ int xcd_tile(int nwg) {
    const int w = blockIdx.x;
    return (w & 7) * (nwg >> 3) + (w >> 3);
}

// Occupancy target of the apply kernels: FP32 forms at <= 128 VGPRs (4 waves
// per SIMD), FP64 at <= 256.
template <class Fmt>
struct Occ {
    static constexpr int waves = 4;
};
template <>
struct Occ<FmtF64> {
    static constexpr int waves = 2;
};

// Single right-hand side.
template <class Fmt, int LOG2L>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Occ<Fmt>::waves))) void k_apply(
    Geo g, GaugeDev d, const typename Prec<Fmt>::V *__restrict__ in, typename Prec<Fmt>::V *__restrict__ out,
    int ntiles, int gamma5, double mass, Epi<typename Prec<Fmt>::V> ep) {
    const int tile = xcd_tile(gridDim.x);
    if (tile >= ntiles) return;
    int p, h, c, t, x1, x2, x3;
    if (!tile_site<LOG2L>(g, tile, threadIdx.x, p, h, c, t, x1, x2, x3)) return;
    site_apply<Fmt, LOG2L>(g, d, in, out, p, h, c, t, x1, x2, x3, mass, gamma5, ep, 0, 0);
}

// Time-column form (L = 2^LOG2L): a lane owns one spatial site (one copy)
// and walks TC consecutive time slices, so psi(t-1), psi(t), psi(t+1) of its
// column -- a whole slice apart in memory, far beyond reach of the L2 once
// every site of a slice is in flight -- are touched by the same lane within
// a few hundred cycles and come from its CU's caches.  Lanes alternate the
// spatial parity sp = (x1+x2+x3) mod 2 every copy pair, so the spatial
// neighbours of a lane are the own sites of its wave-mates.  Right-hand sides
// run over the grid: launch item = (rhs, lane block), rhs outermost.
template <class Fmt, int LOG2L, int TC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Occ<Fmt>::waves))) void k_apply_tcol(
    Geo g, GaugeDev d, const typename Prec<Fmt>::V *__restrict__ in, typename Prec<Fmt>::V *__restrict__ out,
    long stride, int nrhs, int nblk_per_rhs, int gamma5, const double *__restrict__ masses, double mass0,
    Epi<typename Prec<Fmt>::V> ep) {
    constexpr int L = 1 << LOG2L, Lh = L / 2, L3h = L * L * L / 2;
    const int item = xcd_tile(gridDim.x);
    const int j = item / nblk_per_rhs;
    if (j >= nrhs) return;
    const int gid = (item - j * nblk_per_rhs) * 256 + threadIdx.x;
    const int c = gid & 1;
    const int sp = (gid >> 1) & 1;
    const int r = gid >> 2;
    const int hs = r % L3h;
    const int b = r / L3h;
    if (b * TC >= g.T) return;
    const int x1 = hs / (Lh * L);
    const int x2 = (hs / Lh) & (L - 1);
    const int x3 = 2 * (hs & (Lh - 1)) + ((sp + x1 + x2) & 1);
    const double m = masses ? masses[j] : mass0;
    const typename Prec<Fmt>::V *inj = in + j * stride;
    typename Prec<Fmt>::V *outj = out + j * stride;
#pragma nounroll
    for (int k = 0; k < TC; k++) {
        const int t = b * TC + k;
        const int p = (t + sp) & 1;
        const int h = t * L3h + hs;
        // opaque spatial coordinates: the neighbour indices are recomputed per
        // slice rather than held (and spilled) across the loop
        int cj_ = c, x1j = x1, x2j = x2, x3j = x3;
        asm volatile("" : "+v"(cj_), "+v"(x1j), "+v"(x2j), "+v"(x3j));
        site_apply<Fmt, LOG2L>(g, d, inj, outj, p, h, cj_, t, x1j, x2j, x3j, m, gamma5, ep, j, j * stride);
    }
}

// nrhs right-hand sides, each with its own mass (lattices without a
// power-of-two L): every lane applies all of them to its site in turn.
template <class Fmt, int LOG2L>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Occ<Fmt>::waves))) void k_apply_multi(
    Geo g, GaugeDev d, const typename Prec<Fmt>::V *__restrict__ in, typename Prec<Fmt>::V *__restrict__ out,
    long stride, int nrhs, int ntiles, int gamma5, const double *__restrict__ masses, double mass0,
    Epi<typename Prec<Fmt>::V> ep) {
    const int tile = xcd_tile(gridDim.x);
    if (tile >= ntiles) return;
    int p, h, c, t, x1, x2, x3;
    if (!tile_site<LOG2L>(g, tile, threadIdx.x, p, h, c, t, x1, x2, x3)) return;
#pragma nounroll
    for (int j = 0; j < nrhs; j++) {
        const double m = masses ? masses[j] : mass0;
        // opaque copies of the gauge pointers and coordinates: keeps the
        // compiler from hoisting loop-invariant loads and indices (and spilling)
        GaugeDev dj = d;
        asm volatile("" : "+s"(dj.link64), "+s"(dj.link32), "+s"(dj.linkbf_a), "+s"(dj.linkbf_b));
        asm volatile("" : "+s"(dj.phase32), "+s"(dj.clov64), "+s"(dj.clov32));
        int pj = p, hj = h, cj_ = c, tj = t, x1j = x1, x2j = x2, x3j = x3;
        asm volatile("" : "+v"(pj), "+v"(hj), "+v"(cj_), "+v"(tj), "+v"(x1j), "+v"(x2j), "+v"(x3j));
        site_apply<Fmt, LOG2L>(g, dj, in + j * stride, out + j * stride, pj, hj, cj_, tj, x1j, x2j, x3j, m, gamma5, ep,
                               j, j * stride);
    }
}

// Time-marching form (L = 2^LOG2L >= 8).  A workgroup owns RX1 x RX2 rows
// (x1, x2) of the spatial lattice -- a row is the L sites of x3 times the two
// copies, 2L lanes -- and one segment of TB time slices, which it walks in
// order.  Every iteration loads one slice: the x3 neighbours lie in the same
// wave and the x1 / x2 neighbours in sibling waves that load the same lines at
// the same time, so they come from L1 / L2 instead of HBM.  The time hops are
// carried in registers: iteration s loads psi(s) and the link V(s-1, 0) once,
// completes site s-1 with its forward time hop and starts site s with its
// backward time hop (from the projected psi(s-1) kept from the last iteration).
// The running sum is -2 (SW + 4 + m) psi + hops, so the result is -1/2 of it.
template <class R, class V>
__device__ __forceinline__ void finish_site(const Geo &g, V *__restrict__ out, const Epi<V> &ep, int j, long joff, int p,
                                            int h, int c, int gamma5, cx<R> acc[12]) {
    const R s5 = gamma5 ? R(-1) : R(1);
#pragma unroll
    for (int k = 0; k < 12; k++) {
        acc[k] = scale(acc[k], R(-0.5));
        if (k >= 6) acc[k] = scale(acc[k], s5);
    }
    apply_epilogue<R, V>(g, ep, j, joff, p, h, c, acc);
    SpinorIO<R>::store(out, g, p, h, c, acc);
}

// Exchange of one value with another lane of the wave (LDS crossbar, no memory access).
__device__ __forceinline__ float lane_get(int src, float v) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
__device__ __forceinline__ double lane_get(int src, double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Both x3 hops of a site through the wave (L <= 32, so the 2L lanes of an x3
// row -- lane = 2 x3 + copy -- lie in one wave): every lane sends the
// projected (1 - g3) psi(x) to its backward neighbour and V(x,3)^H (1 + g3) psi(x),
// formed with its own link, to its forward neighbour; a hop across the x3
// boundary lands on the other copy.  No spinor or backward link is loaded.
template <class Fmt, int LOG2L>
__device__ __forceinline__ void hop_x3_wave(const Geo &g, const GaugeDev &d, int p, int h, int c, int x3,
                                            const cx<typename Prec<Fmt>::R> v[12],
                                            cx<typename Prec<Fmt>::R> acc[12]) {
    using R = typename Prec<Fmt>::R;
    constexpr int L = 1 << LOG2L;
    static_assert(L <= 32, "an x3 row must fit in one wave");
    const int lane = threadIdx.x & 63;
    const int rowbase = lane & ~(2 * L - 1);
    const int src_f = x3 < L - 1 ? lane + 2 : rowbase + (1 - c);                // site x + 3
    const int src_b = x3 > 0 ? lane - 2 : rowbase + 2 * (L - 1) + (1 - c);      // site x - 3
    Link<R> Lk;
    Fmt::load(d, g, p, 3, h, c ? R(-1) : R(1), Lk);  // V(x,3) of this lane's copy
    {
        cx<R> hh[6], gg[6];
        project<3, 1>(v, hh);
        link_mul<Fmt, true>(Lk, hh, gg);
#pragma unroll
        for (int i = 0; i < 6; i++) hh[i] = {lane_get(src_b, gg[i].re), lane_get(src_b, gg[i].im)};
        accumulate<3, 1>(acc, hh);
    }
    {
        cx<R> hh[6], gg[6];
        project<3, -1>(v, gg);
#pragma unroll
        for (int i = 0; i < 6; i++) hh[i] = {lane_get(src_f, gg[i].re), lane_get(src_f, gg[i].im)};
        link_mul<Fmt, false>(Lk, hh, gg);
        accumulate<3, -1>(acc, gg);
    }
}

// One half of hop_pair from memory, with the link already loaded (forward) or
// loaded here (backward).
template <class Fmt, int MU, int LOG2L>
__device__ __forceinline__ void hop_fwd_mem(const Geo &g, const typename Prec<Fmt>::V *__restrict__ in, int p, int c,
                                            int t, int x1, int x2, int x3, const Link<typename Prec<Fmt>::R> &L,
                                            cx<typename Prec<Fmt>::R> acc[12]) {
    using R = typename Prec<Fmt>::R;
    const Hop n = hop_fwd<MU, LOG2L>(g, t, x1, x2, x3);
    cx<R> v[12], hh[6], gg[6];
    SpinorIO<R>::load(in, g, 1 - p, n.h, c ^ n.flip, v);
    project<MU, -1>(v, hh);
    link_mul<Fmt, false>(L, hh, gg);
    accumulate<MU, -1>(acc, gg);
}
template <class Fmt, int MU, int LOG2L>
__device__ __forceinline__ void hop_bwd_mem(const Geo &g, const GaugeDev &d, const typename Prec<Fmt>::V *__restrict__ in,
                                            int p, int c, int t, int x1, int x2, int x3,
                                            cx<typename Prec<Fmt>::R> acc[12]) {
    using R = typename Prec<Fmt>::R;
    const Hop n = hop_bwd<MU, LOG2L>(g, t, x1, x2, x3);
    const int cn = c ^ n.flip;
    Link<R> L;
    Fmt::load(d, g, 1 - p, MU, n.h, cn ? R(-1) : R(1), L);
    cx<R> v[12], hh[6], gg[6];
    SpinorIO<R>::load(in, g, 1 - p, n.h, cn, v);
    project<MU, 1>(v, hh);
    link_mul<Fmt, true>(L, hh, gg);
    accumulate<MU, 1>(acc, gg);
}

template <class Fmt, int LOG2L, int RX1, int RX2, int TB, bool EPI, bool NTC>
__global__ __launch_bounds__(RX1 * RX2 * (2 << LOG2L)) void k_apply_march(
    Geo g, GaugeDev d, const typename Prec<Fmt>::V *__restrict__ in, typename Prec<Fmt>::V *__restrict__ out,
    long stride, int nrhs, int gamma5, const double *__restrict__ masses, double mass0,
    Epi<typename Prec<Fmt>::V> ep) {
    using R = typename Prec<Fmt>::R;
    using V = typename Prec<Fmt>::V;
    constexpr int L = 1 << LOG2L;
    constexpr int N1 = L / RX1, N2 = L / RX2;
    const int nseg = (g.T + TB - 1) / TB;
    const int per_rhs = N1 * N2 * nseg;
    // right-hand side fastest: the workgroups of one tile for all right-hand
    // sides run together on one XCD and share its link and clover lines in L2
    const int item = xcd_tile(gridDim.x);
    const int j = item % nrhs;
    int r = item / nrhs;
    if (r >= per_rhs) return;
    const int tile2 = r % N2;
    r /= N2;
    const int tile1 = r % N1;
    const int seg = r / N1;
    const int lane = threadIdx.x;
    const int c = lane & 1;
    const int x3 = (lane >> 1) & (L - 1);
    const int row = lane >> (LOG2L + 1);
    const int x2_in = row % RX2, x1_in = row / RX2;
    const int x2 = tile2 * RX2 + x2_in;
    const int x1 = tile1 * RX1 + row / RX2;
    const int t0 = seg * TB;
    const int t1 = min(t0 + TB, g.T);
    const double mass = masses ? masses[j] : mass0;
    const R dmu = R(4.0 + mass + ep.shift), dml = R(4.0 + mass - ep.shift);
    // exchange buffer: [x2 forward, x2 backward, x1 forward payload][half-spinor component][lane]
    __shared__ cx<R> xch[3][6][RX1 * RX2 * (2 << LOG2L)];
    const typename Prec<Fmt>::V *inj = in + j * stride;
    typename Prec<Fmt>::V *outj = out + j * stride;
    const long joff = j * stride;
    const int xs = x1 + x2 + x3;
    const R tsign = g.time_bc < 0 ? R(-1) : R(1);
    const R csg = c ? R(-1) : R(1);

    // prologue: projected psi(t0 - 1) for the backward time hop into t0
    cx<R> hb[6];
    {
        const int tp = t0 == 0 ? g.T - 1 : t0 - 1;
        cx<R> v[12];
        SpinorIO<R>::load(inj, g, (tp + xs) & 1, pair_index<LOG2L>(g, tp, x1, x2, x3), c, v);
        project<0, 1>(v, hb);
        if (t0 == 0) {
#pragma unroll
            for (int k = 0; k < 6; k++) hb[k] = scale(hb[k], tsign);
        }
    }
    cx<R> acc[12];
#pragma unroll
    for (int k = 0; k < 12; k++) acc[k] = {R(0), R(0)};
#pragma nounroll
    for (int s = t0; s <= t1; s++) {
        const int ts = s == g.T ? 0 : s;
        const int tm = s == 0 ? g.T - 1 : s - 1;
        const int ps = (ts + xs) & 1, pm = (tm + xs) & 1;
        const int hs = pair_index<LOG2L>(g, ts, x1, x2, x3), hm = pair_index<LOG2L>(g, tm, x1, x2, x3);
        cx<R> v[12];
        SpinorIO<R>::load(inj, g, ps, hs, c, v);
        Link<R> Lt;  // V(s-1, 0) at the lane's spatial site
        Fmt::load(d, g, pm, 0, hm, csg, Lt);
        if (s > t0) {
            // forward time hop of site s-1: (1 - g0) V(s-1,0) psi(s); then site s-1 is complete
            cx<R> hf[6], gf[6];
            project<0, -1>(v, hf);
            if (s == g.T) {
#pragma unroll
                for (int k = 0; k < 6; k++) hf[k] = scale(hf[k], tsign);
            }
            link_mul<Fmt, false>(Lt, hf, gf);
            accumulate<0, -1>(acc, gf);
            if constexpr (EPI) {
                finish_site<R, V>(g, outj, ep, j, joff, pm, hm, c, gamma5, acc);
            } else {
                // no epilogue: the result is -1/2 acc, times g5
                const R s5 = gamma5 ? R(-1) : R(1);
#pragma unroll
                for (int k = 0; k < 12; k++) acc[k] = scale(acc[k], k < 6 ? R(-0.5) : R(-0.5) * s5);
                SpinorIO<R>::store(outj, g, pm, hm, c, acc);
            }
        }
        if (s < t1) {
            // site s: backward time hop (scaled by -1/2 so that the final -2
            // restores it), local term, then the spatial hops
#pragma unroll
            for (int k = 0; k < 12; k++) acc[k] = {R(0), R(0)};
            {
                cx<R> gb[6];
                link_mul<Fmt, true>(Lt, hb, gb);
                accumulate<0, 1>(acc, gb);
            }
#pragma unroll
            for (int k = 0; k < 12; k++) acc[k] = scale(acc[k], R(-0.5));
            pin(acc);
            clover_add<R, NTC>(d, g, ps, hs, c, v, acc);
#pragma unroll
            for (int k = 0; k < 12; k++) acc[k] = scale(acc[k] + scale(v[k], k < 6 ? dmu : dml), R(-2));
            project<0, 1>(v, hb);
            pin(acc);
            // opaque coordinates: recomputed per slice rather than held across the loop
            int cj_ = c, x1j = x1, x2j = x2, x3j = x3;
            asm volatile("" : "+v"(cj_), "+v"(x1j), "+v"(x2j), "+v"(x3j));
            if constexpr (LOG2L <= 5) {
                hop_x3_wave<Fmt, LOG2L>(g, d, ps, hs, cj_, x3j, v, acc);
            } else {
                hop_pair<Fmt, 3, LOG2L>(g, d, inj, ps, hs, cj_, ts, x1j, x2j, x3j, acc);
            }
            pin(acc);
            // x2 hops: each lane publishes (1 - g2) psi(x) and V(x,2)^H (1 + g2) psi(x)
            // in LDS, and (1 - g1) psi(x) for the x1 forward hop; neighbours
            // inside the workgroup's tile read them, rows on the tile's faces
            // fetch from memory
            Link<R> L2;
            Fmt::load(d, g, ps, 2, hs, csg, L2);
            {
                cx<R> hh[6], gg[6];
                project<2, -1>(v, hh);
#pragma unroll
                for (int i = 0; i < 6; i++) xch[0][i][lane] = hh[i];
                project<2, 1>(v, hh);
                link_mul<Fmt, true>(L2, hh, gg);
#pragma unroll
                for (int i = 0; i < 6; i++) xch[1][i][lane] = gg[i];
                project<1, -1>(v, hh);
#pragma unroll
                for (int i = 0; i < 6; i++) xch[2][i][lane] = hh[i];
            }
            __syncthreads();
            if (x2_in + 1 < RX2) {
                cx<R> hh[6], gg[6];
#pragma unroll
                for (int i = 0; i < 6; i++) hh[i] = xch[0][i][lane + 2 * L];
                link_mul<Fmt, false>(L2, hh, gg);
                accumulate<2, -1>(acc, gg);
            } else {
                hop_fwd_mem<Fmt, 2, LOG2L>(g, inj, ps, cj_, ts, x1j, x2j, x3j, L2, acc);
            }
            pin(acc);
            if (x2_in > 0) {
                cx<R> gg[6];
#pragma unroll
                for (int i = 0; i < 6; i++) gg[i] = xch[1][i][lane - 2 * L];
                accumulate<2, 1>(acc, gg);
            } else {
                hop_bwd_mem<Fmt, 2, LOG2L>(g, d, inj, ps, cj_, ts, x1j, x2j, x3j, acc);
            }
            pin(acc);
            {
                // x1 forward hop: (1 - g1) V(x,1) psi(x+1); the row x1+1 is RX2 rows on
                Link<R> L1;
                Fmt::load(d, g, ps, 1, hs, csg, L1);
                if (x1_in + 1 < RX1) {
                    cx<R> hh[6], gg[6];
#pragma unroll
                    for (int i = 0; i < 6; i++) hh[i] = xch[2][i][lane + RX2 * 2 * L];
                    link_mul<Fmt, false>(L1, hh, gg);
                    accumulate<1, -1>(acc, gg);
                } else {
                    hop_fwd_mem<Fmt, 1, LOG2L>(g, inj, ps, cj_, ts, x1j, x2j, x3j, L1, acc);
                }
            }
            pin(acc);
            __syncthreads();  // the exchange buffer is rewritten in the next slice
            hop_bwd_mem<Fmt, 1, LOG2L>(g, d, inj, ps, cj_, ts, x1j, x2j, x3j, acc);
            pin(acc);
        }
    }
}

// Multi-RHS form of the time-marching kernel: every lane applies NR
// right-hand sides to its site, so each link and clover word it loads serves
// NR spinors (the loads of the gauge field per right-hand side, and their
// bytes, fall by NR).  The sweep is that of k_apply_march; the exchange
// buffer holds the NR payloads of every lane.  Launch item = (tile, group of
// NR right-hand sides), groups fastest, so the groups of one tile run
// together on one XCD and share the remaining gauge reads in its L2.
template <class Fmt, int MU, int LOG2L, int NR>
__device__ __forceinline__ void hop_fwd_mem_nr(const Geo &g, const typename Prec<Fmt>::V *__restrict__ in, long stride,
                                               int p, int c, int t, int x1, int x2, int x3,
                                               const Link<typename Prec<Fmt>::R> &Lk,
                                               cx<typename Prec<Fmt>::R> acc[NR][12]) {
    using R = typename Prec<Fmt>::R;
    const Hop n = hop_fwd<MU, LOG2L>(g, t, x1, x2, x3);
#pragma unroll
    for (int r = 0; r < NR; r++) {
        cx<R> v[12], hh[6], gg[6];
        SpinorIO<R>::load(in + r * stride, g, 1 - p, n.h, c ^ n.flip, v);
        project<MU, -1>(v, hh);
        link_mul<Fmt, false>(Lk, hh, gg);
        accumulate<MU, -1>(acc[r], gg);
    }
}
template <class Fmt, int MU, int LOG2L, int NR>
__device__ __forceinline__ void hop_bwd_mem_nr(const Geo &g, const GaugeDev &d, const typename Prec<Fmt>::V *__restrict__ in,
                                               long stride, int p, int c, int t, int x1, int x2, int x3,
                                               cx<typename Prec<Fmt>::R> acc[NR][12]) {
    using R = typename Prec<Fmt>::R;
    const Hop n = hop_bwd<MU, LOG2L>(g, t, x1, x2, x3);
    const int cn = c ^ n.flip;
    Link<R> Lk;
    Fmt::load(d, g, 1 - p, MU, n.h, cn ? R(-1) : R(1), Lk);
#pragma unroll
    for (int r = 0; r < NR; r++) {
        cx<R> v[12], hh[6], gg[6];
        SpinorIO<R>::load(in + r * stride, g, 1 - p, n.h, cn, v);
        project<MU, 1>(v, hh);
        link_mul<Fmt, true>(Lk, hh, gg);
        accumulate<MU, 1>(acc[r], gg);
    }
}

template <class R, int NR>
__device__ __forceinline__ void pin_nr(cx<R> acc[NR][12]) {
#pragma unroll
    for (int r = 0; r < NR; r++) pin(acc[r]);
}

template <class Fmt, int LOG2L, int RX1, int RX2, int TB, int NR, bool EPI>
__device__ __forceinline__ void march_nr_item(const Geo &g, const GaugeDev &d,
                                              const typename Prec<Fmt>::V *__restrict__ in,
                                              typename Prec<Fmt>::V *__restrict__ out, long stride, int ngrp,
                                              int gamma5, const double *__restrict__ masses, double mass0,
                                              const Epi<typename Prec<Fmt>::V> &ep, int item, int blocked);

template <class Fmt, int LOG2L, int RX1, int RX2, int TB, int NR, bool EPI, bool PERSIST>
__global__ __launch_bounds__(RX1 * RX2 * (2 << LOG2L)) void k_apply_march_nr(
    Geo g, GaugeDev d, const typename Prec<Fmt>::V *__restrict__ in, typename Prec<Fmt>::V *__restrict__ out,
    long stride, int ngrp, int gamma5, const double *__restrict__ masses, double mass0,
    Epi<typename Prec<Fmt>::V> ep, int nitems, int blocked) {
    if constexpr (!PERSIST) {
        march_nr_item<Fmt, LOG2L, RX1, RX2, TB, NR, EPI>(g, d, in, out, stride, ngrp, gamma5, masses, mass0, ep,
                                                         xcd_tile(gridDim.x), blocked);
    } else {
        // persistent: workgroup w stays on XCD w mod 8 and walks that XCD's
        // contiguous range of items (nitems is a multiple of 8) with the
        // XCD's other workgroups; every thread of a workgroup takes the same
        // items, so the slice barriers inside stay uniform
        const int w = blockIdx.x, x = w & 7, nloc = gridDim.x >> 3;
        const int per_xcd = nitems >> 3;
        for (int k = w >> 3; k < per_xcd; k += nloc)
            march_nr_item<Fmt, LOG2L, RX1, RX2, TB, NR, EPI>(g, d, in, out, stride, ngrp, gamma5, masses, mass0,
                                                             ep, x * per_xcd + k, blocked);
    }
}

template <class Fmt, int LOG2L, int RX1, int RX2, int TB, int NR, bool EPI>
__device__ __forceinline__ void march_nr_item(const Geo &g, const GaugeDev &d,
                                              const typename Prec<Fmt>::V *__restrict__ in,
                                              typename Prec<Fmt>::V *__restrict__ out, long stride, int ngrp,
                                              int gamma5, const double *__restrict__ masses, double mass0,
                                              const Epi<typename Prec<Fmt>::V> &ep, int item, int blocked) {
    using R = typename Prec<Fmt>::R;
    using V = typename Prec<Fmt>::V;
    constexpr int L = 1 << LOG2L;
    constexpr int N1 = L / RX1, N2 = L / RX2;
    constexpr int LANES = RX1 * RX2 * (2 << LOG2L);
    const int nseg = (g.T + TB - 1) / TB;
    const int per_grp = N1 * N2 * nseg;
    int grp, r_;
    if (blocked == 2) {
        // group slowest: an XCD's contiguous range of items is one group's
        // tiles, so the workgroups in flight on it are neighbouring tiles of
        // one group and share their face rows in L2
        grp = item / per_grp;
        r_ = item - grp * per_grp;
        if (grp >= ngrp) return;
    } else {
        grp = item % ngrp;
        r_ = item / ngrp;
        if (r_ >= per_grp) return;
    }
    int tile1, tile2, seg;
    if (blocked == 1 && N1 % 2 == 0 && N2 % 4 == 0) {
        // consecutive tiles (which run together on one XCD) form 2 x 4 blocks of
        // tiles in (x1, x2), so more of their faces are shared inside the block
        const int l = r_ % 8;
        int b = r_ / 8;
        tile2 = (b % (N2 / 4)) * 4 + (l & 3);
        b /= N2 / 4;
        tile1 = (b % (N1 / 2)) * 2 + (l >> 2);
        seg = b / (N1 / 2);
    } else {
        tile2 = r_ % N2;
        tile1 = (r_ / N2) % N1;
        seg = r_ / (N1 * N2);
    }
    const int lane = threadIdx.x;
    const int c = lane & 1;
    const int x3 = (lane >> 1) & (L - 1);
    const int row = lane >> (LOG2L + 1);
    const int x2_in = row % RX2, x1_in = row / RX2;
    const int x2 = tile2 * RX2 + x2_in;
    const int x1 = tile1 * RX1 + x1_in;
    const int t0 = seg * TB;
    const int t1 = min(t0 + TB, g.T);
    const int j0 = grp * NR;
    R dmu[NR], dml[NR];
#pragma unroll
    for (int r = 0; r < NR; r++) {
        const double mass = masses ? masses[j0 + r] : mass0;
        dmu[r] = R(4.0 + mass + ep.shift);
        dml[r] = R(4.0 + mass - ep.shift);
    }
    __shared__ cx<R> xch[NR][3][6][LANES];
    const V *inj = in + j0 * stride;
    V *outj = out + j0 * stride;
    const int xs = x1 + x2 + x3;
    const R tsign = g.time_bc < 0 ? R(-1) : R(1);
    const R csg = c ? R(-1) : R(1);

    cx<R> hb[NR][6];
    {
        const int tp = t0 == 0 ? g.T - 1 : t0 - 1;
        const int pp = (tp + xs) & 1, hp = pair_index<LOG2L>(g, tp, x1, x2, x3);
#pragma unroll
        for (int r = 0; r < NR; r++) {
            cx<R> v[12];
            SpinorIO<R>::load(inj + r * stride, g, pp, hp, c, v);
            project<0, 1>(v, hb[r]);
            if (t0 == 0) {
#pragma unroll
                for (int k = 0; k < 6; k++) hb[r][k] = scale(hb[r][k], tsign);
            }
        }
    }
    cx<R> acc[NR][12];
#pragma unroll
    for (int r = 0; r < NR; r++)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[r][k] = {R(0), R(0)};
#pragma nounroll
    for (int s = t0; s <= t1; s++) {
        const int ts = s == g.T ? 0 : s;
        const int tm = s == 0 ? g.T - 1 : s - 1;
        const int ps = (ts + xs) & 1, pm = (tm + xs) & 1;
        const int hs = pair_index<LOG2L>(g, ts, x1, x2, x3), hm = pair_index<LOG2L>(g, tm, x1, x2, x3);
        cx<R> v[NR][12];
#pragma unroll
        for (int r = 0; r < NR; r++) SpinorIO<R>::load(inj + r * stride, g, ps, hs, c, v[r]);
        Link<R> Lt;  // V(s-1, 0) at the lane's spatial site
        Fmt::load(d, g, pm, 0, hm, csg, Lt);
        if (s > t0) {
            // forward time hop of site s-1, then site s-1 is complete
#pragma unroll
            for (int r = 0; r < NR; r++) {
                cx<R> hf[6], gf[6];
                project<0, -1>(v[r], hf);
                if (s == g.T) {
#pragma unroll
                    for (int k = 0; k < 6; k++) hf[k] = scale(hf[k], tsign);
                }
                link_mul<Fmt, false>(Lt, hf, gf);
                accumulate<0, -1>(acc[r], gf);
                if constexpr (EPI) {
                    finish_site<R, V>(g, outj + r * stride, ep, j0 + r, (long)(j0 + r) * stride, pm, hm, c, gamma5,
                                      acc[r]);
                } else {
                    const R s5 = gamma5 ? R(-1) : R(1);
#pragma unroll
                    for (int k = 0; k < 12; k++) acc[r][k] = scale(acc[r][k], k < 6 ? R(-0.5) : R(-0.5) * s5);
                    SpinorIO<R>::store(outj + r * stride, g, pm, hm, c, acc[r]);
                }
            }
        }
        if (s < t1) {
#pragma unroll
            for (int r = 0; r < NR; r++) {
#pragma unroll
                for (int k = 0; k < 12; k++) acc[r][k] = {R(0), R(0)};
                cx<R> gb[6];
                link_mul<Fmt, true>(Lt, hb[r], gb);
                accumulate<0, 1>(acc[r], gb);
#pragma unroll
                for (int k = 0; k < 12; k++) acc[r][k] = scale(acc[r][k], R(-0.5));
            }
            pin_nr<R, NR>(acc);
            // clover: each chirality block loaded once, applied to every right-hand side
#pragma unroll
            for (int b = 0; b < 2; b++) {
                R dg[6];
                cx<R> o[15];
                CloverIO<R>::template load<false>(d, g, ps, hs, b, dg, o);
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    cx<R> u[6], w[6];
#pragma unroll
                    for (int a = 0; a < 3; a++) {
                        const cx<R> c0 = v[r][6 * b + a], c1 = v[r][6 * b + 3 + a];
                        u[a] = c ? mk(-c1.im, -c1.re) : c0;
                        u[3 + a] = c ? mk(c0.im, c0.re) : c1;
                    }
                    herm6_mul(dg, o, u, w);
#pragma unroll
                    for (int a = 0; a < 3; a++) {
                        const cx<R> q0 = c ? mk(w[3 + a].im, w[3 + a].re) : w[a];
                        const cx<R> q1 = c ? mk(-w[a].im, -w[a].re) : w[3 + a];
                        acc[r][6 * b + a] = acc[r][6 * b + a] + q0;
                        acc[r][6 * b + 3 + a] = acc[r][6 * b + 3 + a] + q1;
                    }
                }
                pin_nr<R, NR>(acc);
            }
#pragma unroll
            for (int r = 0; r < NR; r++) {
#pragma unroll
                for (int k = 0; k < 12; k++)
                    acc[r][k] = scale(acc[r][k] + scale(v[r][k], k < 6 ? dmu[r] : dml[r]), R(-2));
                project<0, 1>(v[r], hb[r]);
            }
            pin_nr<R, NR>(acc);
            int cj_ = c, x1j = x1, x2j = x2, x3j = x3;
            asm volatile("" : "+v"(cj_), "+v"(x1j), "+v"(x2j), "+v"(x3j));
            {
                // x3 hops through the wave, one link for every right-hand side
                static_assert(LOG2L <= 5, "an x3 row must fit in one wave");
                const int wl = threadIdx.x & 63;
                const int rowbase = wl & ~(2 * L - 1);
                const int src_f = x3j < L - 1 ? wl + 2 : rowbase + (1 - cj_);
                const int src_b = x3j > 0 ? wl - 2 : rowbase + 2 * (L - 1) + (1 - cj_);
                Link<R> L3;
                Fmt::load(d, g, ps, 3, hs, csg, L3);
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    cx<R> hh[6], gg[6];
                    project<3, 1>(v[r], hh);
                    link_mul<Fmt, true>(L3, hh, gg);
#pragma unroll
                    for (int i = 0; i < 6; i++) hh[i] = {lane_get(src_b, gg[i].re), lane_get(src_b, gg[i].im)};
                    accumulate<3, 1>(acc[r], hh);
                    project<3, -1>(v[r], gg);
#pragma unroll
                    for (int i = 0; i < 6; i++) hh[i] = {lane_get(src_f, gg[i].re), lane_get(src_f, gg[i].im)};
                    link_mul<Fmt, false>(L3, hh, gg);
                    accumulate<3, -1>(acc[r], gg);
                }
            }
            pin_nr<R, NR>(acc);
            Link<R> L2;
            Fmt::load(d, g, ps, 2, hs, csg, L2);
#pragma unroll
            for (int r = 0; r < NR; r++) {
                cx<R> hh[6], gg[6];
                project<2, -1>(v[r], hh);
#pragma unroll
                for (int i = 0; i < 6; i++) xch[r][0][i][lane] = hh[i];
                project<2, 1>(v[r], hh);
                link_mul<Fmt, true>(L2, hh, gg);
#pragma unroll
                for (int i = 0; i < 6; i++) xch[r][1][i][lane] = gg[i];
                project<1, -1>(v[r], hh);
#pragma unroll
                for (int i = 0; i < 6; i++) xch[r][2][i][lane] = hh[i];
            }
            __syncthreads();
            if (x2_in + 1 < RX2) {
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    cx<R> hh[6], gg[6];
#pragma unroll
                    for (int i = 0; i < 6; i++) hh[i] = xch[r][0][i][lane + 2 * L];
                    link_mul<Fmt, false>(L2, hh, gg);
                    accumulate<2, -1>(acc[r], gg);
                }
            } else {
                hop_fwd_mem_nr<Fmt, 2, LOG2L, NR>(g, inj, stride, ps, cj_, ts, x1j, x2j, x3j, L2, acc);
            }
            pin_nr<R, NR>(acc);
            if (x2_in > 0) {
#pragma unroll
                for (int r = 0; r < NR; r++) {
                    cx<R> gg[6];
#pragma unroll
                    for (int i = 0; i < 6; i++) gg[i] = xch[r][1][i][lane - 2 * L];
                    accumulate<2, 1>(acc[r], gg);
                }
            } else {
                hop_bwd_mem_nr<Fmt, 2, LOG2L, NR>(g, d, inj, stride, ps, cj_, ts, x1j, x2j, x3j, acc);
            }
            pin_nr<R, NR>(acc);
            {
                Link<R> L1;
                Fmt::load(d, g, ps, 1, hs, csg, L1);
                if (x1_in + 1 < RX1) {
#pragma unroll
                    for (int r = 0; r < NR; r++) {
                        cx<R> hh[6], gg[6];
#pragma unroll
                        for (int i = 0; i < 6; i++) hh[i] = xch[r][2][i][lane + RX2 * 2 * L];
                        link_mul<Fmt, false>(L1, hh, gg);
                        accumulate<1, -1>(acc[r], gg);
                    }
                } else {
                    hop_fwd_mem_nr<Fmt, 1, LOG2L, NR>(g, inj, stride, ps, cj_, ts, x1j, x2j, x3j, L1, acc);
                }
            }
            pin_nr<R, NR>(acc);
            __syncthreads();  // the exchange buffer is rewritten in the next slice
            hop_bwd_mem_nr<Fmt, 1, LOG2L, NR>(g, d, inj, stride, ps, cj_, ts, x1j, x2j, x3j, acc);
            pin_nr<R, NR>(acc);
        }
    }
}

// rows of a marching workgroup: 1024 lanes for the FP32 forms, 512 for FP64
template <class Fmt>
struct March {
    static constexpr int lanes = 1024;
};
template <>
struct March<FmtF64> {
    static constexpr int lanes = 512;
};
constexpr int march_rows(int lanes, int log2l) { return lanes >> (log2l + 1); }
constexpr int march_rx1(int rows) { return rows >= 64 ? 8 : rows >= 16 ? 4 : 2; }

// Multi-RHS launch of the time-marching form over right-hand sides
// [j_begin, j_begin + NR * ngrp): pointers, masses and epilogue operands are
// shifted to the first of them.
template <class V>
static Epi<V> shift_epi(const Epi<V> &ep, long off, int j_begin, bool fp64) {
    Epi<V> e = ep;
    if (e.y) e.y += off;
    if (e.z) e.z += off;
    if (e.w) e.w += off;
    if (e.ew) e.ew = fp64 ? (const void *)((const double *)e.ew + j_begin) : (const void *)((const float *)e.ew + j_begin);
    return e;
}

template <class Fmt, int LOG2L, int RX1, int RX2, int TB, int NR, bool PERSIST = false>
static void launch_march_nr(const Geo &g, const GaugeDev &d, const ApplyArgs &a, const Epi<typename Prec<Fmt>::V> &ep,
                            int j_begin, int ngrp, hipStream_t s, int blocked = 0) {
    using V = typename Prec<Fmt>::V;
    constexpr int LANES = RX1 * RX2 * (2 << LOG2L);
    const long st = a.stride / (long)sizeof(V);
    const long off = (long)j_begin * st;
    const Epi<V> e = shift_epi(ep, off, j_begin, sizeof(typename Prec<Fmt>::R) == 8);
    const int nseg = (g.T + TB - 1) / TB;
    const long items = (long)((1 << LOG2L) / RX1) * ((1 << LOG2L) / RX2) * nseg * ngrp;
    const int nitems = (int)((items + 7) / 8 * 8);
    // persistent: two 256-lane workgroups per CU of the 256-CU chip
    const int nwg = PERSIST ? std::min(nitems, 512) : nitems;
    const double *m = a.masses_dev ? a.masses_dev + j_begin : nullptr;
    if (e.on)
        hipLaunchKernelGGL((k_apply_march_nr<Fmt, LOG2L, RX1, RX2, TB, NR, true, PERSIST>), dim3(nwg), dim3(LANES), 0,
                           s, g, d, (const V *)a.in + off, (V *)a.out + off, st, ngrp, a.gamma5, m, a.mass0, e, nitems,
                           blocked);
    else
        hipLaunchKernelGGL((k_apply_march_nr<Fmt, LOG2L, RX1, RX2, TB, NR, false, PERSIST>), dim3(nwg), dim3(LANES), 0,
                           s, g, d, (const V *)a.in + off, (V *)a.out + off, st, ngrp, a.gamma5, m, a.mass0, e, nitems,
                           blocked);
}

// Single-RHS-per-lane time-marching launch over right-hand sides [j_begin, j_begin + n).
template <class Fmt, int LOG2L>
static void launch_march_1(const Geo &g, const GaugeDev &d, const ApplyArgs &a, const Epi<typename Prec<Fmt>::V> &ep,
                           int j_begin, int n, hipStream_t s) {
    using V = typename Prec<Fmt>::V;
    constexpr int rows = march_rows(March<Fmt>::lanes, LOG2L);
    constexpr int RX1 = march_rx1(rows), RX2 = rows / RX1;
    constexpr int TB = 8;
    static_assert(RX1 * RX2 * (2 << LOG2L) == March<Fmt>::lanes, "march tile");
    const long st = a.stride / (long)sizeof(V);
    const long off = (long)j_begin * st;
    const Epi<V> e = shift_epi(ep, off, j_begin, sizeof(typename Prec<Fmt>::R) == 8);
    const int nseg = (g.T + TB - 1) / TB;
    const long items = (long)((1 << LOG2L) / RX1) * ((1 << LOG2L) / RX2) * nseg * n;
    const int nwg = (int)((items + 7) / 8 * 8);
    const double *m = a.masses_dev ? a.masses_dev + j_begin : nullptr;
    const bool one = n == 1;
    if constexpr (LOG2L <= 5) {
        // few workgroups per CU in the default tiling: 256-lane workgroups
        // (2 x 4 rows at L = 16, 4 x 4 at L = 8 marching 2 slices; 2 x 2 rows
        // marching 16 slices at L = 32) give 4 to 16 times as many, with the
        // same arithmetic per site, so the same bits.  Used below one default
        // workgroup per CU, and for the FP32 forms below four (16^4, 16
        // right-hand sides: 0.157 against 0.175 ms; 32^4, one: 0.206 against
        // 0.224 ms; FP64 is slower with them)
        constexpr int rows_s = march_rows(256, LOG2L);
        constexpr int RX1s = march_rx1(rows_s), RX2s = rows_s / RX1s;
        constexpr int TBs = LOG2L == 5 ? 16 : 2;
        static_assert(RX1s * RX2s * (2 << LOG2L) == 256, "small march tile");
        if (nwg < (std::is_same<Fmt, FmtF64>::value ? 256 : 1024)) {
            const int nseg_s = (g.T + TBs - 1) / TBs;
            const long items_s = (long)((1 << LOG2L) / RX1s) * ((1 << LOG2L) / RX2s) * nseg_s * n;
            const int nwg_s = (int)((items_s + 7) / 8 * 8);
            auto go_s = [&](auto kern) {
                hipLaunchKernelGGL(kern, dim3(nwg_s), dim3(256), 0, s, g, d, (const V *)a.in + off,
                                   (V *)a.out + off, st, n, a.gamma5, m, a.mass0, e);
            };
            if (e.on) {
                if (one) go_s(k_apply_march<Fmt, LOG2L, RX1s, RX2s, TBs, true, true>);
                else go_s(k_apply_march<Fmt, LOG2L, RX1s, RX2s, TBs, true, false>);
            } else {
                if (one) go_s(k_apply_march<Fmt, LOG2L, RX1s, RX2s, TBs, false, true>);
                else go_s(k_apply_march<Fmt, LOG2L, RX1s, RX2s, TBs, false, false>);
            }
            return;
        }
    }
    // epilogue compiled in only where used; clover streamed only when one right-hand side reads it
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(nwg), dim3(March<Fmt>::lanes), 0, s, g, d, (const V *)a.in + off,
                           (V *)a.out + off, st, n, a.gamma5, m, a.mass0, e);
    };
    if (e.on) {
        if (one) go(k_apply_march<Fmt, LOG2L, RX1, RX2, TB, true, true>);
        else go(k_apply_march<Fmt, LOG2L, RX1, RX2, TB, true, false>);
    } else {
        if (one) go(k_apply_march<Fmt, LOG2L, RX1, RX2, TB, false, true>);
        else go(k_apply_march<Fmt, LOG2L, RX1, RX2, TB, false, false>);
    }
}

// Schedules of a multi-RHS launch of the FP32 forms at L = 32 (the tuner's candidates):
//   0: one right-hand side per lane, 1024-lane workgroups of 4 x 4 rows, 8 slices;
//   1: two per lane, 512 lanes, 2 x 4 rows, 8 slices;   2: two per lane, 4 x 2 rows, 8 slices;
//   3: two per lane, 2 x 4 rows, 16 slices;             4: four per lane, 256 lanes, 2 x 2 rows, 8 slices;
//   5: two per lane, 256 lanes, 2 x 2 rows, 8 slices;   6: two per lane, 256 lanes, 2 x 2 rows, 16 slices;
//   7: schedule 6 as one persistent launch (512 workgroups walking the items);
//   8, 9: schedules 6, 7 with the tiles dealt in 2 x 4 blocks;
//   10, 11, 12: schedules 6, 7, 2 with the groups of right-hand sides slowest
//   (each XCD runs neighbouring tiles of one group).
// (256-lane workgroups leave room for two per CU, so one computes while the
// other waits at its slice barrier.)  Right-hand sides beyond the last full
// group of a schedule go to schedule 0.
constexpr int march_nr_of(int sched) { return sched == 0 ? 1 : sched == 4 ? 4 : 2; }

template <class Fmt>
static void launch_march_sched32(int sched, const Geo &g, const GaugeDev &d, const ApplyArgs &a,
                                 const Epi<typename Prec<Fmt>::V> &ep, hipStream_t s) {
    const int nr = march_nr_of(sched);
    const int ngrp = a.nrhs / nr;
    const int done = ngrp * nr;
    if (ngrp > 0) {
        switch (sched) {
            case 1: launch_march_nr<Fmt, 5, 2, 4, 8, 2>(g, d, a, ep, 0, ngrp, s); break;
            case 2: launch_march_nr<Fmt, 5, 4, 2, 8, 2>(g, d, a, ep, 0, ngrp, s); break;
            case 3: launch_march_nr<Fmt, 5, 2, 4, 16, 2>(g, d, a, ep, 0, ngrp, s); break;
            case 4: launch_march_nr<Fmt, 5, 2, 2, 8, 4>(g, d, a, ep, 0, ngrp, s); break;
            case 5: launch_march_nr<Fmt, 5, 2, 2, 8, 2>(g, d, a, ep, 0, ngrp, s); break;
            case 6: launch_march_nr<Fmt, 5, 2, 2, 16, 2>(g, d, a, ep, 0, ngrp, s); break;
            case 7: launch_march_nr<Fmt, 5, 2, 2, 16, 2, true>(g, d, a, ep, 0, ngrp, s); break;
            case 8: launch_march_nr<Fmt, 5, 2, 2, 16, 2>(g, d, a, ep, 0, ngrp, s, 1); break;
            case 9: launch_march_nr<Fmt, 5, 2, 2, 16, 2, true>(g, d, a, ep, 0, ngrp, s, 1); break;
            case 10: launch_march_nr<Fmt, 5, 2, 2, 16, 2>(g, d, a, ep, 0, ngrp, s, 2); break;
            case 11: launch_march_nr<Fmt, 5, 2, 2, 16, 2, true>(g, d, a, ep, 0, ngrp, s, 2); break;
            case 12: launch_march_nr<Fmt, 5, 4, 2, 8, 2>(g, d, a, ep, 0, ngrp, s, 2); break;
            default: launch_march_1<Fmt, 5>(g, d, a, ep, 0, a.nrhs, s); return;
        }
    }
    if (done < a.nrhs) launch_march_1<Fmt, 5>(g, d, a, ep, done, a.nrhs - done, s);
}

template <class Fmt, int LOG2L>
static void launch_apply_l(const Geo &g, const GaugeDev &d, const ApplyArgs &a, hipStream_t s, cstar_prec prec) {
    using V = typename Prec<Fmt>::V;
    Epi<V> ep{(const V *)a.y, (const V *)a.z, (float)a.ea, (float)a.eb, (float)a.ec, a.ea, a.eb, a.ec,
              (a.y || a.z || a.w || a.ea != 1.0) ? 1 : 0, (const V *)a.w, a.ew, a.shift};
    const long st = a.stride / (long)sizeof(V);
    const int ntiles = (4 * g.Vh + 255) / 256;
    if constexpr (LOG2L == 5 && !std::is_same<Fmt, FmtF64>::value) {
        if (a.nrhs > 1) {
            auto go = [&](int sched) { launch_march_sched32<Fmt>(sched, g, d, a, ep, s); };
            go(march_schedule(g, prec, a, s, go));
            return;
        }
    }
    if constexpr (LOG2L >= 3) {
        launch_march_1<Fmt, LOG2L>(g, d, a, ep, 0, a.nrhs, s);
        return;
    }
    if constexpr (LOG2L >= 2) {
        // lanes per right-hand side: 2 L^3 (sites x copies) x T / TC
        const long lanes = 2L * (1L << (3 * LOG2L)) * (g.T % 4 == 0 ? g.T / 4 : g.T / 2);
        const int nblk = (int)((lanes + 255) / 256);
        const long items = (long)nblk * a.nrhs;
        const int nwg = (int)((items + 7) / 8 * 8);
        if (g.T % 4 == 0)
            hipLaunchKernelGGL((k_apply_tcol<Fmt, (LOG2L >= 2 ? LOG2L : 2), 4>), dim3(nwg), dim3(256), 0, s, g, d,
                               (const V *)a.in, (V *)a.out, st, a.nrhs, nblk, a.gamma5, a.masses_dev, a.mass0, ep);
        else
            hipLaunchKernelGGL((k_apply_tcol<Fmt, (LOG2L >= 2 ? LOG2L : 2), 2>), dim3(nwg), dim3(256), 0, s, g, d,
                               (const V *)a.in, (V *)a.out, st, a.nrhs, nblk, a.gamma5, a.masses_dev, a.mass0, ep);
        return;
    }
    const int nwg = (ntiles + 7) / 8 * 8;
    if (a.nrhs == 1 && !a.masses_dev)
        hipLaunchKernelGGL((k_apply<Fmt, LOG2L>), dim3(nwg), dim3(256), 0, s, g, d, (const V *)a.in, (V *)a.out,
                           ntiles, a.gamma5, a.mass0, ep);
    else
        hipLaunchKernelGGL((k_apply_multi<Fmt, LOG2L>), dim3(nwg), dim3(256), 0, s, g, d, (const V *)a.in,
                           (V *)a.out, st, a.nrhs, ntiles, a.gamma5, a.masses_dev, a.mass0, ep);
}

template <class Fmt>
static void launch_apply_t(const Geo &g, const GaugeDev &d, const ApplyArgs &a, hipStream_t s, cstar_prec prec) {
    switch (g.L) {
        case 4: launch_apply_l<Fmt, 2>(g, d, a, s, prec); break;
        case 8: launch_apply_l<Fmt, 3>(g, d, a, s, prec); break;
        case 16: launch_apply_l<Fmt, 4>(g, d, a, s, prec); break;
        case 32: launch_apply_l<Fmt, 5>(g, d, a, s, prec); break;
        case 64: launch_apply_l<Fmt, 6>(g, d, a, s, prec); break;
        default: launch_apply_l<Fmt, 0>(g, d, a, s, prec); break;
    }
}

hipError_t launch_apply(const Geo &g, const GaugeDev &d, cstar_prec prec, const ApplyArgs &a, hipStream_t s) {
    if (prec == CSTAR_FP64)
        launch_apply_t<FmtF64>(g, d, a, s, prec);
    else if (prec == CSTAR_FP32)
        launch_apply_t<FmtF32>(g, d, a, s, prec);
    else
        launch_apply_t<FmtBF16>(g, d, a, s, prec);
    return hipGetLastError();
}

// ---------------------------------------------------------------- link packing
__device__ __forceinline__ unsigned bf16_bits(double v) {
    // FP64 -> nearest FP32 -> round-to-nearest-even on the upper 16 bits
    const unsigned u = __float_as_uint((float)v);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ unsigned bf16_pair(double lo, double hi) { return bf16_bits(lo) | (bf16_bits(hi) << 16); }

__global__ void k_pack_links(Geo g, const double *__restrict__ su3, const double *__restrict__ theta, double q,
                             GaugeDev d) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 2 * g.Vh * 4) return;
    const int mu = gid & 3;
    const int pair = gid >> 2;
    const int p = pair >= g.Vh;
    const int h = pair - p * g.Vh;
    int t, x1, x2, x3;
    decode(g, p, h, t, x1, x2, x3);
    const long lex = ((long)(t * g.L + x1) * g.L + x2) * g.L + x3;
    const double *u = su3 + (lex * 4 + mu) * 18;
    const double th = theta[lex * 4 + mu];
    const double phi = q * th;
    double sn, cs;
    sincos(phi, &sn, &cs);
    const long base9 = (long)(p * 4 + mu) * 9;
    for (int r = 0; r < 9; r++) {
        const double re = u[2 * r], im = u[2 * r + 1];
        d.link64[(base9 + r) * g.Vh + h] = make_double2(cs * re - sn * im, cs * im + sn * re);
    }
    const long base3 = (long)(p * 4 + mu) * 3;
    for (int k = 0; k < 3; k++)
        d.link32[(base3 + k) * g.Vh + h] = make_float4((float)u[4 * k], (float)u[4 * k + 1], (float)u[4 * k + 2],
                                                       (float)u[4 * k + 3]);
    const long i = (long)(p * 4 + mu) * g.Vh + h;
    d.linkbf_a[i] = make_uint4(bf16_pair(u[0], u[1]), bf16_pair(u[2], u[3]), bf16_pair(u[4], u[5]),
                               bf16_pair(u[6], u[7]));
    d.linkbf_b[i] = make_uint2(bf16_pair(u[8], u[9]), bf16_pair(u[10], u[11]));
    d.phase32[i] = make_float2((float)cs, (float)sn);
}

hipError_t launch_pack_links(const Geo &g, const double *su3, const double *theta, double q, GaugeDev &d,
                             hipStream_t s) {
    const int n = 2 * g.Vh * 4;
    hipLaunchKernelGGL(k_pack_links, dim3((n + 255) / 256), dim3(256), 0, s, g, su3, theta, q, d);
    return hipGetLastError();
}

// ---------------------------------------------------------------- clover
// A point of the doubled lattice in pair form: physical coordinates + copy index.
struct Pt {
    int t, x1, x2, x3, c;
};

__device__ __forceinline__ Pt step(const Geo &g, Pt a, int mu, int dir) {
    int *x = mu == 0 ? &a.t : mu == 1 ? &a.x1 : mu == 2 ? &a.x2 : &a.x3;
    const int ext = mu == 0 ? g.T : g.L;
    *x += dir;
    if (*x == ext || *x < 0) {
        *x = (*x + ext) % ext;
        if (mu) a.c ^= 1;
    }
    return a;
}

// U_e(a, mu) with its U(1) angle on the doubled lattice
__device__ __forceinline__ void load_link64(const Geo &g, const double *su3, const double *theta, Pt a, int mu,
                                            cx<double> U[9], double &th) {
    const long lex = ((long)(a.t * g.L + a.x1) * g.L + a.x2) * g.L + a.x3;
    const double *u = su3 + (lex * 4 + mu) * 18;
    const double s = a.c ? -1.0 : 1.0;
#pragma unroll
    for (int r = 0; r < 9; r++) U[r] = {u[2 * r], s * u[2 * r + 1]};
    th = s * theta[lex * 4 + mu];
}

__device__ __forceinline__ void mm3(const cx<double> A[9], const cx<double> B[9], cx<double> C[9]) {
    cx<double> r[9];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<double> s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; k++) s = s + A[i * 3 + k] * B[k * 3 + j];
            r[i * 3 + j] = s;
        }
#pragma unroll
    for (int i = 0; i < 9; i++) C[i] = r[i];
}
__device__ __forceinline__ void mm3_dag_right(const cx<double> A[9], const cx<double> B[9], cx<double> C[9]) {
    // C = A * B^H
    cx<double> r[9];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) {
            cx<double> s = {0.0, 0.0};
#pragma unroll
            for (int k = 0; k < 3; k++) s = s + A[i * 3 + k] * cj(B[j * 3 + k]);
            r[i * 3 + j] = s;
        }
#pragma unroll
    for (int i = 0; i < 9; i++) C[i] = r[i];
}

// Plaquette leaf starting and ending at x: the loop x -> x+s1 -> ... with
// signed unit steps (mu first, then nu for the same orientation).
__device__ void leaf(const Geo &g, const double *su3, const double *theta, Pt x, const int steps[4], cx<double> P[9],
                     double &ang) {
#pragma unroll
    for (int i = 0; i < 9; i++) P[i] = {0.0, 0.0};
    P[0] = P[4] = P[8] = {1.0, 0.0};
    ang = 0.0;
    Pt y = x;
    for (int k = 0; k < 4; k++) {
        const int mu = (steps[k] > 0 ? steps[k] : -steps[k]) - 1;
        cx<double> U[9];
        double th;
        if (steps[k] > 0) {
            load_link64(g, su3, theta, y, mu, U, th);
            mm3(P, U, P);
            ang += th;
            y = step(g, y, mu, +1);
        } else {
            y = step(g, y, mu, -1);
            load_link64(g, su3, theta, y, mu, U, th);
            mm3_dag_right(P, U, P);
            ang -= th;
        }
    }
}

// One thread per physical site: F_{mu nu} for the six planes, the two
// chirality blocks of (i/2) sum_{mu<nu} sigma_{mu nu} F_{mu nu} in closed
// form for this basis:
//   sigma_{0k} = diag(s_k, -s_k),  sigma_{jk} = -eps_{jkl} diag(s_l, s_l),
//   block(X) = (i/2) [[X3, X1 - i X2], [X1 + i X2, -X3]],
//   upper X = (F01 - F23, F02 + F13, F03 - F12), lower X = (-F01 - F23, -F02 + F13, -F03 - F12).
__global__ void k_clover(Geo g, const double *__restrict__ su3, const double *__restrict__ theta, double q,
                         double csw_su3, double csw_u1, GaugeDev d, double *__restrict__ norm_partial) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    double nrm = 0.0;
    if (gid < 2 * g.Vh) {
        const int p = gid >= g.Vh;
        const int h = gid - p * g.Vh;
        Pt x;
        decode(g, p, h, x.t, x.x1, x.x2, x.x3);
        x.c = 0;
        cx<double> F[6][9];
        const int planes[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
        for (int pl = 0; pl < 6; pl++) {
            const int a = planes[pl][0] + 1, b = planes[pl][1] + 1;
            const int lv[4][4] = {{a, b, -a, -b}, {b, -a, -b, a}, {-a, -b, a, b}, {-b, a, b, -a}};
            cx<double> Qs[9];
            for (int i = 0; i < 9; i++) Qs[i] = {0.0, 0.0};
            double ssum = 0.0;
            for (int l = 0; l < 4; l++) {
                cx<double> P[9];
                double ang;
                leaf(g, su3, theta, x, lv[l], P, ang);
                for (int i = 0; i < 9; i++) Qs[i] = Qs[i] + P[i];
                ssum += sin(ang);
            }
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    // (Q - Q^H)/8
                    const cx<double> qij = Qs[i * 3 + j], qji = Qs[j * 3 + i];
                    cx<double> f = {csw_su3 * (qij.re - qji.re) / 8.0, csw_su3 * (qij.im + qji.im) / 8.0};
                    if (i == j) f.im += q * csw_u1 * 0.25 * ssum;
                    F[pl][i * 3 + j] = f;
                }
        }
        for (int blk = 0; blk < 2; blk++) {
            const double s0 = blk == 0 ? 1.0 : -1.0;
            cx<double> X[3][9];
            for (int i = 0; i < 9; i++) {
                X[0][i] = scale(F[0][i], s0) - F[5][i];
                X[1][i] = scale(F[1][i], s0) + F[4][i];
                X[2][i] = scale(F[2][i], s0) - F[3][i];
            }
            // M (6x6), index s*3 + colour; M = (i/2) [[X3, X1 - i X2],[X1 + i X2, -X3]]
            cx<double> M[6][6];
            for (int i = 0; i < 3; i++)
                for (int j = 0; j < 3; j++) {
                    const cx<double> x1v = X[0][i * 3 + j], x2v = X[1][i * 3 + j], x3v = X[2][i * 3 + j];
                    M[i][j] = scale(mul_i(x3v), 0.5);
                    M[3 + i][3 + j] = scale(mul_i(x3v), -0.5);
                    M[i][3 + j] = scale(mul_i(x1v - mul_i(x2v)), 0.5);
                    M[3 + i][j] = scale(mul_i(x1v + mul_i(x2v)), 0.5);
                }
            double rowsum_max = 0.0, frob = 0.0;
            for (int i = 0; i < 6; i++) {
                double rs = 0.0;
                for (int j = 0; j < 6; j++) {
                    const double m2 = M[i][j].re * M[i][j].re + M[i][j].im * M[i][j].im;
                    rs += sqrt(m2);
                    frob += m2;
                }
                rowsum_max = fmax(rowsum_max, rs);
            }
            nrm = fmax(nrm, fmin(rowsum_max, sqrt(frob)));
            double2 *q64 = d.clov64 + (long)(p * 36 + blk * 18) * g.Vh + h;
            float *tmp = nullptr;
            (void)tmp;
            double re36[36];
            for (int i = 0; i < 6; i++) re36[i] = M[i][i].re;
            for (int i = 1; i < 6; i++)
                for (int j = 0; j < i; j++) {
                    const int k = i * (i - 1) / 2 + j;
                    re36[6 + 2 * k] = M[i][j].re;
                    re36[7 + 2 * k] = M[i][j].im;
                }
            for (int k = 0; k < 18; k++) q64[(long)k * g.Vh] = make_double2(re36[2 * k], re36[2 * k + 1]);
            float4 *q32 = d.clov32 + (long)(p * 18 + blk * 9) * g.Vh + h;
            for (int k = 0; k < 9; k++)
                q32[(long)k * g.Vh] = make_float4((float)re36[4 * k], (float)re36[4 * k + 1], (float)re36[4 * k + 2],
                                                  (float)re36[4 * k + 3]);
        }
    }
    // block max of the per-site norm bound
    __shared__ double red[256];
    red[threadIdx.x] = nrm;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) norm_partial[blockIdx.x] = red[0];
}

int clover_norm_blocks(const Geo &g) { return (2 * g.Vh + 255) / 256; }

hipError_t launch_clover(const Geo &g, const double *su3, const double *theta, double q, double csw_su3,
                         double csw_u1, GaugeDev &d, double *norm_partial, hipStream_t s) {
    hipLaunchKernelGGL(k_clover, dim3(clover_norm_blocks(g)), dim3(256), 0, s, g, su3, theta, q, csw_su3, csw_u1, d,
                       norm_partial);
    return hipGetLastError();
}

// ---------------------------------------------------------------- layout conversion
// canonical [T][2L][L][L][4][3] complex  <->  native (see cstar.h)
template <class R>
__global__ void k_pack_spinor(Geo g, const void *__restrict__ src, void *__restrict__ dst, int nrhs, int unpack) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= 4 * g.Vh) return;
    const int c = gid & 1;
    const int pair = gid >> 1;
    const int p = pair >= g.Vh;
    const int h = pair - p * g.Vh;
    int t, x1, x2, x3;
    decode(g, p, h, t, x1, x2, x3);
    const long site = ((long)(t * 2 * g.L + x1 + c * g.L) * g.L + x2) * g.L + x3;
    const long nsite = 4L * g.Vh;
    using V = typename SpinorIO<R>::vec;
    const long nvec = (long)(sizeof(R) == 8 ? 12 : 6) * nsite;  // native vector entries per rhs
    for (int j = 0; j < nrhs; j++) {
        cx<R> v[12];
        if (!unpack) {
            const cx<R> *s = (const cx<R> *)src + (j * nsite + site) * 12;
#pragma unroll
            for (int k = 0; k < 12; k++) v[k] = s[k];
            SpinorIO<R>::store((V *)dst + j * nvec, g, p, h, c, v);
        } else {
            SpinorIO<R>::load((const V *)src + j * nvec, g, p, h, c, v);
            cx<R> *s = (cx<R> *)dst + (j * nsite + site) * 12;
#pragma unroll
            for (int k = 0; k < 12; k++) s[k] = v[k];
        }
    }
}

hipError_t launch_pack_spinor(const Geo &g, cstar_prec prec, int nrhs, void *canon, void *native, int unpack,
                              hipStream_t s) {
    const int n = 4 * g.Vh;
    const dim3 grd((n + 255) / 256), blk(256);
    if (prec == CSTAR_FP64) {
        if (!unpack)
            hipLaunchKernelGGL(k_pack_spinor<double>, grd, blk, 0, s, g, canon, native, nrhs, 0);
        else
            hipLaunchKernelGGL(k_pack_spinor<double>, grd, blk, 0, s, g, (const void *)native, (void *)canon, nrhs, 1);
    } else {
        if (!unpack)
            hipLaunchKernelGGL(k_pack_spinor<float>, grd, blk, 0, s, g, canon, native, nrhs, 0);
        else
            hipLaunchKernelGGL(k_pack_spinor<float>, grd, blk, 0, s, g, (const void *)native, (void *)canon, nrhs, 1);
    }
    return hipGetLastError();
}

long n_cplx(const Geo &g) { return 4L * g.Vh * 12; }

}  // namespace cstar
