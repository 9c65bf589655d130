// HIP kernels of the gauge-covariant preconditioner network (FP32 arithmetic).
//
// A layer maps Cin channels of spinor fields to Cout channels:
//   out_a(x) = sum_b sum_p W[a][b][p] (T_p in_b)(x),
// W[a][b][p] a complex 4x4 matrix on spin, T_0 = 1 and, for p = 1 + 2 mu + d,
//   d = 0: (T_p psi)(x) = V(x,mu) psi(x+mu),   d = 1: (T_p psi)(x) = V(x-mu,mu)^H psi(x-mu)
// on the x-doubled C* lattice (a hop across the x1/x2/x3 boundary lands on the
// other copy, whose links are the conjugates; a hop across the time boundary
// takes the fermion time phase).  The transports commute with spin matrices
// and are unitary, so the input gradient of a layer is again a layer:
//   grad in_b = sum_p' sum_a W[a][b][rev p']^H T_p' grad out_a.
//
// Activations: FP32 native spinors (float4 [p][6][Vh][2]), channel c of a
// block at c * cs float4.  Weights: FP32 [Cout][Cin][9][4][4] complex,
// interleaved (re, im).  Links: the FP32 rows with the FP32 quark phase.
#include "lattice_dev.h"
#include "nn_kernels.h"

namespace cstar {

namespace {

constexpr int NPATH = 9;

__device__ __forceinline__ int nn_xcd_tile(int nwg) {
    const int w = blockIdx.x;
    return (w & 7) * (nwg >> 3) + (w >> 3);
}

// (T_P psi) at the lane's site (pair (p, h), copy c, coordinates t, x1, x2, x3)
template <int P>
__device__ __forceinline__ void transport(const Geo &g, const GaugeDev &d, const float4 *__restrict__ in, int p, int h,
                                          int c, int t, int x1, int x2, int x3, cx<float> o[12]) {
    if constexpr (P == 0) {
        SpinorIO<float>::load(in, g, p, h, c, o);
    } else {
        constexpr int MU = (P - 1) / 2;
        constexpr bool FWD = ((P - 1) & 1) == 0;
        const Hop n = FWD ? hop_fwd<MU, 0>(g, t, x1, x2, x3) : hop_bwd<MU, 0>(g, t, x1, x2, x3);
        const int cn = c ^ n.flip;
        Link<float> L;
        if (FWD)
            FmtF32::load(d, g, p, MU, h, c ? -1.f : 1.f, L);
        else
            FmtF32::load(d, g, 1 - p, MU, n.h, cn ? -1.f : 1.f, L);
        cx<float> v[12];
        SpinorIO<float>::load(in, g, 1 - p, n.h, cn, v);
        if (MU == 0 && n.tw && g.time_bc < 0) {
#pragma unroll
            for (int k = 0; k < 12; k++) v[k] = scale(v[k], -1.f);
        }
        link_mul<FmtF32, !FWD>(L, v, o);
        link_mul<FmtF32, !FWD>(L, v + 6, o + 6);
    }
}

// Materialise the accumulators here: the loads and arithmetic of one path
// cannot be interleaved with the next path's, which bounds the live registers.
template <int CB>
__device__ __forceinline__ void pin_acc(cx<float> acc[CB][12]) {
#pragma unroll
    for (int a = 0; a < CB; a++)
#pragma unroll
        for (int k = 0; k < 12; k++) asm volatile("" : "+v"(acc[a][k].re), "+v"(acc[a][k].im));
}

// acc[a] += W[a0+a][b][P] (T_P in_b) for the CB output channels of this pass;
// Ws: the workgroup's weights [CB][CIN][9][4][4] complex in LDS (uniform reads)
template <int P, int CIN, int CB>
__device__ __forceinline__ void layer_path(const Geo &g, const GaugeDev &d, const float4 *__restrict__ inb, int p,
                                           int h, int c, int t, int x1, int x2, int x3, const float *Ws, int b,
                                           cx<float> acc[CB][12]) {
    cx<float> tv[12];
    transport<P>(g, d, inb, p, h, c, t, x1, x2, x3, tv);
#pragma unroll
    for (int a = 0; a < CB; a++) {
        // row s of the 4x4 block: two float4 = four complex entries (s, s')
        const float4 *w = reinterpret_cast<const float4 *>(Ws + ((a * CIN + b) * NPATH + P) * 32);
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const float4 w01 = w[2 * s], w23 = w[2 * s + 1];
            const cx<float> ws[4] = {{w01.x, w01.y}, {w01.z, w01.w}, {w23.x, w23.y}, {w23.z, w23.w}};
#pragma unroll
            for (int sp = 0; sp < 4; sp++)
#pragma unroll
                for (int col = 0; col < 3; col++)
                    acc[a][s * 3 + col] = cmac(acc[a][s * 3 + col], ws[sp], tv[sp * 3 + col]);
        }
    }
}

// grid: x = site tiles of 256 lanes (lane = one site of the doubled lattice),
// y = blocks of CB output channels
template <int CIN, int CB>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_nn_layer(Geo g, GaugeDev d, const float4 *__restrict__ in, long cs_in,
                                                  float4 *__restrict__ out, long cs_out, const float *__restrict__ W,
                                                  int cout, int ntiles) {
    __shared__ float4 Ws4[CB * CIN * NPATH * 8];
    const int a0 = blockIdx.y * CB;
    {
        const float4 *src = reinterpret_cast<const float4 *>(W + (long)a0 * CIN * NPATH * 32);
        const int nw = (cout - a0 < CB ? cout - a0 : CB) * CIN * NPATH * 8;
        for (int i = threadIdx.x; i < CB * CIN * NPATH * 8; i += 256) Ws4[i] = i < nw ? src[i] : make_float4(0, 0, 0, 0);
    }
    __syncthreads();
    const float *Ws = reinterpret_cast<const float *>(Ws4);
    const int tile = nn_xcd_tile(gridDim.x);
    if (tile >= ntiles) return;
    const int gid = tile * 256 + threadIdx.x;
    if (gid >= 4 * g.Vh) return;
    const int c = gid & 1;
    const int q = gid >> 1;
    const int p = q >= g.Vh;
    const int h = q - p * g.Vh;
    int t, x1, x2, x3;
    decode(g, p, h, t, x1, x2, x3);
    cx<float> acc[CB][12];
#pragma unroll
    for (int a = 0; a < CB; a++)
#pragma unroll
        for (int k = 0; k < 12; k++) acc[a][k] = {0.f, 0.f};
#pragma nounroll
    for (int b = 0; b < CIN; b++) {
        const float4 *inb = in + b * cs_in;
        layer_path<0, CIN, CB>(g, d, inb, p, h, c, t, x1, x2, x3, Ws, b, acc);
        pin_acc<CB>(acc);
        layer_path<1, CIN, CB>(g, d, inb, p, h, c, t, x1, x2, x3, Ws, b, acc);
        pin_acc<CB>(acc);
        layer_path<2, CIN, CB>(g, d, inb, p, h, c, t, x1, x2, x3, Ws, b, acc);
        pin_acc<CB>(acc);
        layer_path<3, CIN, CB>(g, d, inb, p, h, c, t, x1, x2, x3, Ws, b, acc);
        pin_acc<CB>(acc);
        layer_path<4, CIN, CB>(g, d, inb, p, h, c, t, x1, x2, x3, Ws, b, acc);
        pin_acc<CB>(acc);
        layer_path<5, CIN, CB>(g, d, inb, p, h, c, t, x1, x2, x3, Ws, b, acc);
        pin_acc<CB>(acc);
        layer_path<6, CIN, CB>(g, d, inb, p, h, c, t, x1, x2, x3, Ws, b, acc);
        pin_acc<CB>(acc);
        layer_path<7, CIN, CB>(g, d, inb, p, h, c, t, x1, x2, x3, Ws, b, acc);
        pin_acc<CB>(acc);
        layer_path<8, CIN, CB>(g, d, inb, p, h, c, t, x1, x2, x3, Ws, b, acc);
        pin_acc<CB>(acc);
    }
#pragma unroll
    for (int a = 0; a < CB; a++)
        if (a0 + a < cout) SpinorIO<float>::store(out + (a0 + a) * cs_out, g, p, h, c, acc[a]);
}

// Weight gradient of one layer:
//   gW[a][b][p][s][s'] = sum_x sum_col gout_a(x)[s][col] conj((T_p in_b)(x)[s'][col]).
// grid: x = NB workgroups striding over the sites, y = (b, p), z = blocks of CB
// output channels.  Lanes sum their sites in FP32; the workgroup sums its
// lanes in FP64 in a fixed order and writes one partial per slot.
template <int P, int CB>
__device__ __forceinline__ void wgrad_sites(const Geo &g, const GaugeDev &d, const float4 *__restrict__ inb,
                                            const float4 *__restrict__ gout, long cs_g, int a0, int cout,
                                            cx<float> acc[CB][16]) {
    const int nlanes = gridDim.x * 256;
    for (int gid = blockIdx.x * 256 + threadIdx.x; gid < 4 * g.Vh; gid += nlanes) {
        const int c = gid & 1;
        const int q = gid >> 1;
        const int p = q >= g.Vh;
        const int h = q - p * g.Vh;
        int t, x1, x2, x3;
        decode(g, p, h, t, x1, x2, x3);
        cx<float> tv[12];
        transport<P>(g, d, inb, p, h, c, t, x1, x2, x3, tv);
#pragma unroll
        for (int a = 0; a < CB; a++) {
            if (a0 + a >= cout) break;
            cx<float> gv[12];
            SpinorIO<float>::load(gout + (a0 + a) * cs_g, g, p, h, c, gv);
#pragma unroll
            for (int s = 0; s < 4; s++)
#pragma unroll
                for (int sp = 0; sp < 4; sp++)
#pragma unroll
                    for (int col = 0; col < 3; col++)
                        acc[a][s * 4 + sp] = cmac_conj(acc[a][s * 4 + sp], tv[sp * 3 + col], gv[s * 3 + col]);
        }
    }
}

template <int CB>
__global__ __launch_bounds__(256) void k_nn_wgrad(Geo g, GaugeDev d, const float4 *__restrict__ in, long cs_in,
                                                  int cin, const float4 *__restrict__ gout, long cs_g, int cout,
                                                  double *__restrict__ partial) {
    const int b = blockIdx.y / NPATH;
    const int path = blockIdx.y - b * NPATH;
    const int a0 = blockIdx.z * CB;
    const float4 *inb = in + b * cs_in;
    cx<float> acc[CB][16];
#pragma unroll
    for (int a = 0; a < CB; a++)
#pragma unroll
        for (int k = 0; k < 16; k++) acc[a][k] = {0.f, 0.f};
    switch (path) {
        case 0: wgrad_sites<0, CB>(g, d, inb, gout, cs_g, a0, cout, acc); break;
        case 1: wgrad_sites<1, CB>(g, d, inb, gout, cs_g, a0, cout, acc); break;
        case 2: wgrad_sites<2, CB>(g, d, inb, gout, cs_g, a0, cout, acc); break;
        case 3: wgrad_sites<3, CB>(g, d, inb, gout, cs_g, a0, cout, acc); break;
        case 4: wgrad_sites<4, CB>(g, d, inb, gout, cs_g, a0, cout, acc); break;
        case 5: wgrad_sites<5, CB>(g, d, inb, gout, cs_g, a0, cout, acc); break;
        case 6: wgrad_sites<6, CB>(g, d, inb, gout, cs_g, a0, cout, acc); break;
        case 7: wgrad_sites<7, CB>(g, d, inb, gout, cs_g, a0, cout, acc); break;
        default: wgrad_sites<8, CB>(g, d, inb, gout, cs_g, a0, cout, acc); break;
    }
    // fixed-order FP64 reduction: butterfly within each wave, then the four waves in order
    __shared__ double red[4][CB * 32];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < CB; a++)
#pragma unroll
        for (int k = 0; k < 16; k++) {
            double re = acc[a][k].re, im = acc[a][k].im;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                re += __shfl_xor(re, off, 64);
                im += __shfl_xor(im, off, 64);
            }
            if (lane == 0) {
                red[wv][(a * 16 + k) * 2] = re;
                red[wv][(a * 16 + k) * 2 + 1] = im;
            }
        }
    __syncthreads();
    // partial layout: [blockIdx.x][cout][cin][9][16] complex
    for (int i = threadIdx.x; i < CB * 32; i += 256) {
        const int a = i / 32, r = i - a * 32;
        if (a0 + a >= cout) continue;
        const double v = ((red[0][i] + red[1][i]) + red[2][i]) + red[3][i];
        const long slot = ((long)((a0 + a) * cin + b) * NPATH + path) * 32 + r;
        partial[(long)blockIdx.x * cout * cin * NPATH * 32 + slot] = v;
    }
}

// grad[i] += sum over the NB partials in order
__global__ void k_nn_wgrad_reduce(const double *__restrict__ partial, int nb, long n, double *__restrict__ grad) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < nb; k++) s += partial[(long)k * n + i];
    grad[i] += s;
}

// Weights of the input-gradient pass: Wt[b][a][p] = W[a][b][rev p]^H
__global__ void k_nn_wt(const float *__restrict__ W, int cout, int cin, float *__restrict__ Wt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;  // over cin * cout * 9 * 16
    if (i >= cin * cout * NPATH * 16) return;
    const int e = i & 15, s = e >> 2, sp = e & 3;
    int r = i >> 4;
    const int p = r % NPATH;
    r /= NPATH;
    const int a = r % cout;
    const int b = r / cout;
    const int rp = p == 0 ? 0 : 1 + 2 * ((p - 1) >> 1) + (1 - ((p - 1) & 1));
    // (W^H)[s][sp] = conj(W[sp][s])
    const float *w = W + ((long)(a * cin + b) * NPATH + rp) * 32 + (sp * 4 + s) * 2;
    Wt[(long)i * 2] = w[0];
    Wt[(long)i * 2 + 1] = -w[1];
}

// gout = s (y - x) over n float4 entries (x null: zero); per-block partial of |y - x|^2 in FP64
__global__ __launch_bounds__(256) void k_nn_resid(long n, const float4 *__restrict__ y, const float4 *__restrict__ x,
                                                  float s, float4 *__restrict__ gout, double *__restrict__ partial) {
    double acc = 0.0;
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
        const float4 a = y[i], b = x ? x[i] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float4 r = make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
        acc += (double)r.x * r.x + (double)r.y * r.y + (double)r.z * r.z + (double)r.w * r.w;
        if (gout) gout[i] = make_float4(s * r.x, s * r.y, s * r.z, s * r.w);
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Adam on FP32 weights from an FP64 gradient (bias-corrected step sizes given)
__global__ void k_nn_adam(int n, float *__restrict__ w, const double *__restrict__ grad, float *__restrict__ m,
                          float *__restrict__ v, float b1, float b2, float step, float eps_hat) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = (float)grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= step * mi / (sqrtf(vi) + eps_hat);
}

}  // namespace

hipError_t launch_nn_layer(const Geo &g, const GaugeDev &d, const float4 *in, int cin, float4 *out, int cout,
                           const float *W, hipStream_t s) {
    const long cs = 24L * g.Vh;
    const int ntiles = (4 * g.Vh + 255) / 256;
    const int nwg = (ntiles + 7) / 8 * 8;
    if (cout == 1) {
        if (cin == 8)
            hipLaunchKernelGGL((k_nn_layer<8, 1>), dim3(nwg, 1), dim3(256), 0, s, g, d, in, cs, out, cs, W, cout, ntiles);
        else if (cin == 1)
            hipLaunchKernelGGL((k_nn_layer<1, 1>), dim3(nwg, 1), dim3(256), 0, s, g, d, in, cs, out, cs, W, cout, ntiles);
        else
            return hipErrorInvalidValue;
    } else {
        const int ny = (cout + 3) / 4;
        if (cin == 8)
            hipLaunchKernelGGL((k_nn_layer<8, 4>), dim3(nwg, ny), dim3(256), 0, s, g, d, in, cs, out, cs, W, cout, ntiles);
        else if (cin == 1)
            hipLaunchKernelGGL((k_nn_layer<1, 4>), dim3(nwg, ny), dim3(256), 0, s, g, d, in, cs, out, cs, W, cout, ntiles);
        else
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int nn_wgrad_blocks(const Geo &g) {
    const int ntiles = (4 * g.Vh + 255) / 256;
    return ntiles < 64 ? ntiles : 64;
}

hipError_t launch_nn_wgrad(const Geo &g, const GaugeDev &d, const float4 *in, int cin, const float4 *gout, int cout,
                           double *partial, double *grad, hipStream_t s) {
    const long cs = 24L * g.Vh;
    const int nb = nn_wgrad_blocks(g);
    const int nz = (cout + 1) / 2;
    hipLaunchKernelGGL((k_nn_wgrad<2>), dim3(nb, cin * NPATH, nz), dim3(256), 0, s, g, d, in, cs, cin, gout, cs, cout,
                       partial);
    const long n = (long)cout * cin * NPATH * 32;
    hipLaunchKernelGGL(k_nn_wgrad_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, partial, nb, n, grad);
    return hipGetLastError();
}

hipError_t launch_nn_wt(const float *W, int cout, int cin, float *Wt, hipStream_t s) {
    const int n = cin * cout * NPATH * 16;
    hipLaunchKernelGGL(k_nn_wt, dim3((n + 255) / 256), dim3(256), 0, s, W, cout, cin, Wt);
    return hipGetLastError();
}

int nn_resid_blocks() { return 512; }

hipError_t launch_nn_resid(long n4, const float4 *y, const float4 *x, float scale, float4 *gout, double *partial,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_nn_resid, dim3(nn_resid_blocks()), dim3(256), 0, s, n4, y, x, scale, gout, partial);
    return hipGetLastError();
}

hipError_t launch_nn_adam(int n, float *w, const double *grad, float *m, float *v, float b1, float b2, float step,
                          float eps_hat, hipStream_t s) {
    hipLaunchKernelGGL(k_nn_adam, dim3((n + 255) / 256), dim3(256), 0, s, n, w, grad, m, v, b1, b2, step, eps_hat);
    return hipGetLastError();
}

}  // namespace cstar
