// Vector kernels of the eigensolver on native spinor blocks (gfx950).
//
// An FP64 block holds nv vectors of n complex entries (double2), vector i at
// base + i*ld.  FP32 native vectors (float4 = two complex entries) are only
// touched by the elementwise kernels and the precision conversions.
//
//  * gram: G[i][j] = sum_n conj(V_i[n]) W_j[n] (FP64 matrix cores), one
//    partial matrix per wave, then a fixed-order sum (bit-reproducible); a
//    single pair of vectors (a dot product) by plain coalesced FMAs instead;
//  * combine: Out_j = sum_i V_i C[i][j] (block rotation / projection);
//  * lincomb: y = a x + b y + c z elementwise (real a,b,c), FP64 or FP32;
//  * precision conversion between the FP64 and FP32 native layouts;
//  * Gaussian fill from a counter-based hash.
#include "cstar_internal.h"
#include "blas.h"

namespace cstar {

constexpr int GT = 64;   // max vectors per side of one gram tile

// Gram tile on the FP64 matrix cores: G = V^H W as real products,
//   Re G = Vr^T Wr + Vi^T Wi,  Im G = Vr^T Wi - Vi^T Wr,
// with v_mfma_f64_16x16x4f64 (per instruction D[16x16] += A[16x4] B[4x16];
// lane l supplies A[l%16][l/16] and B[l/16][l%16] and holds
// D[l/16 + 4r][l%16] in register r).  Every wave owns one contiguous range of
// n and reads its operands straight from memory (16 vectors x 4 consecutive
// entries per load), writes one partial matrix, entry e = i nw + j of wave w
// at partial[e * nwv + w]; the partials of an entry are summed in a fixed
// order afterwards, so the result is bit-reproducible.  The number of waves
// grows as the matrix shrinks (as many as the partial buffer holds, at most
// 8192), so that small Gram matrices still keep enough loads in flight.
typedef double d4v __attribute__((ext_vector_type(4)));

template <int TI, int TJ>
__global__ __launch_bounds__(256) void k_gram(const double2 *__restrict__ V, long ldv, int nv,
                                              const double2 *__restrict__ W, long ldw, int nw, long n,
                                              double2 *__restrict__ partial) {
    const int lane = threadIdx.x & 63;
    const int wv = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int nwv = gridDim.x * 4;
    long chunk = (n + nwv - 1) / nwv;
    chunk = (chunk + 7) & ~7L;
    const long k0 = (long)wv * chunk;
    const long k1 = k0 + chunk < n ? k0 + chunk : n;
    const int r = lane & 15, kk = lane >> 4;
    const bool sym = (V == W) && (ldv == ldw) && (nv == nw) && (TI == TJ);
    d4v cre[TI][TJ], cim[TI][TJ];
#pragma unroll
    for (int a = 0; a < TI; a++)
#pragma unroll
        for (int b = 0; b < TJ; b++) {
            cre[a][b] = d4v{0.0, 0.0, 0.0, 0.0};
            cim[a][b] = d4v{0.0, 0.0, 0.0, 0.0};
        }
#pragma unroll 2
    for (long k = k0; k < k1; k += 4) {
        const long kx = k + kk;
        const bool kin = kx < k1;
        double vr[TI], vi[TI], wr[TJ], wi[TJ];
#pragma unroll
        for (int a = 0; a < TI; a++) {
            const int i = a * 16 + r;
            const double2 v = (kin && i < nv) ? V[(long)i * ldv + kx] : make_double2(0.0, 0.0);
            vr[a] = v.x;
            vi[a] = v.y;
        }
#pragma unroll
        for (int b = 0; b < TJ; b++) {
            if (sym) {
                wr[b] = vr[b < TI ? b : 0];
                wi[b] = vi[b < TI ? b : 0];
            } else {
                const int j = b * 16 + r;
                const double2 w = (kin && j < nw) ? W[(long)j * ldw + kx] : make_double2(0.0, 0.0);
                wr[b] = w.x;
                wi[b] = w.y;
            }
        }
#pragma unroll
        for (int a = 0; a < TI; a++)
#pragma unroll
            for (int b = 0; b < TJ; b++) {
                cre[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(vr[a], wr[b], cre[a][b], 0, 0, 0);
                cre[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(vi[a], wi[b], cre[a][b], 0, 0, 0);
                cim[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(vr[a], wi[b], cim[a][b], 0, 0, 0);
                cim[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(-vi[a], wr[b], cim[a][b], 0, 0, 0);
            }
    }
#pragma unroll
    for (int a = 0; a < TI; a++)
#pragma unroll
        for (int b = 0; b < TJ; b++)
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int i = a * 16 + kk + 4 * q, j = b * 16 + r;
                if (i < nv && j < nw)
                    partial[(long)(i * nw + j) * nwv + wv] = make_double2(cre[a][b][q], cim[a][b][q]);
            }
}

// Entry e of the Gram matrix (one workgroup per entry): the nblk partials of
// e, each thread a fixed strided subset in order, then a fixed tree.
__global__ __launch_bounds__(256) void k_gram_reduce(const double2 *__restrict__ partial, int nblk,
                                                     double2 *__restrict__ out) {
    __shared__ double2 red[256];
    const int e = blockIdx.x, t = threadIdx.x;
    double sx = 0.0, sy = 0.0;
    for (int b = t; b < nblk; b += 256) {
        const double2 v = partial[(long)e * nblk + b];
        sx += v.x;
        sy += v.y;
    }
    red[t] = make_double2(sx, sy);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] = make_double2(red[t].x + red[t + w].x, red[t].y + red[t + w].y);
        __syncthreads();
    }
    if (t == 0) out[e] = red[0];
}

// x^H y for one pair of vectors: consecutive lanes read consecutive entries,
// FP64 FMAs in a fixed order per lane, a fixed tree per workgroup, one partial
// per workgroup (reduced by k_gram_reduce as a 1 x 1 matrix).
constexpr int kDotBlocks = 2048;
__global__ __launch_bounds__(256) void k_dot1(const double2 *__restrict__ x, const double2 *__restrict__ y, long n,
                                              double2 *__restrict__ partial) {
    __shared__ double2 red[256];
    const int t = threadIdx.x;
    double sr = 0.0, si = 0.0;
    const long step = (long)gridDim.x * 256;
    long i = (long)blockIdx.x * 256 + t;
    for (; i + step < n; i += 2 * step) {
        const double2 a0 = x[i], b0 = y[i], a1 = x[i + step], b1 = y[i + step];
        sr = fma(a0.x, b0.x, fma(a0.y, b0.y, sr));
        si = fma(a0.x, b0.y, fma(-a0.y, b0.x, si));
        sr = fma(a1.x, b1.x, fma(a1.y, b1.y, sr));
        si = fma(a1.x, b1.y, fma(-a1.y, b1.x, si));
    }
    if (i < n) {
        const double2 a0 = x[i], b0 = y[i];
        sr = fma(a0.x, b0.x, fma(a0.y, b0.y, sr));
        si = fma(a0.x, b0.y, fma(-a0.y, b0.x, si));
    }
    red[t] = make_double2(sr, si);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] = make_double2(red[t].x + red[t + w].x, red[t].y + red[t + w].y);
        __syncthreads();
    }
    if (t == 0) partial[blockIdx.x] = red[0];
}

// x^H y for one pair of FP32 native vectors (float4 = two complex entries),
// accumulated in FP64 in the same fixed order as k_dot1
__global__ __launch_bounds__(256) void k_dot1f(const float4 *__restrict__ x, const float4 *__restrict__ y, long n4,
                                               double2 *__restrict__ partial) {
    __shared__ double2 red[256];
    const int t = threadIdx.x;
    double sr = 0.0, si = 0.0;
    for (long i = (long)blockIdx.x * 256 + t; i < n4; i += (long)gridDim.x * 256) {
        const float4 a = x[i], b = y[i];
        sr = fma((double)a.x, (double)b.x, fma((double)a.y, (double)b.y, sr));
        si = fma((double)a.x, (double)b.y, fma(-(double)a.y, (double)b.x, si));
        sr = fma((double)a.z, (double)b.z, fma((double)a.w, (double)b.w, sr));
        si = fma((double)a.z, (double)b.w, fma(-(double)a.w, (double)b.z, si));
    }
    red[t] = make_double2(sr, si);
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] = make_double2(red[t].x + red[t + w].x, red[t].y + red[t + w].y);
        __syncthreads();
    }
    if (t == 0) partial[blockIdx.x] = red[0];
}

hipError_t launch_dot32(const float4 *x, const float4 *y, long n4, double2 *partial, double2 *out_dev,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_dot1f, dim3(kDotBlocks), dim3(256), 0, s, x, y, n4, partial);
    hipLaunchKernelGGL(k_gram_reduce, dim3(1), dim3(256), 0, s, partial, kDotBlocks, out_dev);
    return hipGetLastError();
}

int gram_blocks() { return 1024; }
size_t gram_partial_bytes() { return (size_t)gram_blocks() * GT * GT * sizeof(double2); }

// waves of a Gram launch for an nv x nw matrix: as many as the partial buffer
// holds, at most 8192, a multiple of 4 (four waves per workgroup)
static int gram_waves(int nv, int nw) {
    const long cap = (long)gram_blocks() * GT * GT / ((long)nv * nw);
    return (int)(std::min<long>(8192, cap) & ~3L);
}

template <int TI>
static void launch_gram_ti(int tj, int nblk, hipStream_t s, const double2 *V, long ldv, int nv, const double2 *W,
                           long ldw, int nw, long n, double2 *partial) {
    const dim3 grd(nblk / 4), blk(256);
    switch (tj) {
        case 1: hipLaunchKernelGGL((k_gram<TI, 1>), grd, blk, 0, s, V, ldv, nv, W, ldw, nw, n, partial); break;
        case 2: hipLaunchKernelGGL((k_gram<TI, 2>), grd, blk, 0, s, V, ldv, nv, W, ldw, nw, n, partial); break;
        case 3: hipLaunchKernelGGL((k_gram<TI, 3>), grd, blk, 0, s, V, ldv, nv, W, ldw, nw, n, partial); break;
        default: hipLaunchKernelGGL((k_gram<TI, 4>), grd, blk, 0, s, V, ldv, nv, W, ldw, nw, n, partial); break;
    }
}

hipError_t launch_gram(const double2 *V, long ldv, int nv, const double2 *W, long ldw, int nw, long n,
                       double2 *partial, double2 *out_dev, hipStream_t s) {
    if (nv > GT || nw > GT || nv < 1 || nw < 1) return hipErrorInvalidValue;
    if (nv == 1 && nw == 1) {
        hipLaunchKernelGGL(k_dot1, dim3(kDotBlocks), dim3(256), 0, s, V, W, n, partial);
        hipLaunchKernelGGL(k_gram_reduce, dim3(1), dim3(256), 0, s, partial, kDotBlocks, out_dev);
        return hipGetLastError();
    }
    const int nblk = gram_waves(nv, nw);  // partial matrices = waves of the launch
    const int ti = (nv + 15) / 16, tj = (nw + 15) / 16;
    switch (ti) {
        case 1: launch_gram_ti<1>(tj, nblk, s, V, ldv, nv, W, ldw, nw, n, partial); break;
        case 2: launch_gram_ti<2>(tj, nblk, s, V, ldv, nv, W, ldw, nw, n, partial); break;
        case 3: launch_gram_ti<3>(tj, nblk, s, V, ldv, nv, W, ldw, nw, n, partial); break;
        default: launch_gram_ti<4>(tj, nblk, s, V, ldv, nv, W, ldw, nw, n, partial); break;
    }
    hipLaunchKernelGGL(k_gram_reduce, dim3(nv * nw), dim3(256), 0, s, partial, nblk, out_dev);
    return hipGetLastError();
}

// Out_j[n] = beta * Out_j[n] + sum_i V_i[n] C[i*ldc + j]  (i < nv, j < no), C in device memory.
// CJ output columns per pass (chosen >= no so that V is read once).
template <int CJ>
__global__ __launch_bounds__(256) void k_combine(const double2 *__restrict__ V, long ldv, int nv,
                                                 const double2 *__restrict__ C, int ldc, double2 *__restrict__ O,
                                                 long ldo, int no, long n, double beta) {
    __shared__ double2 sC[128 * CJ];
    const int j0 = blockIdx.y * CJ;
    for (int e = threadIdx.x; e < nv * CJ; e += blockDim.x) {
        const int i = e / CJ, jj = e % CJ;
        sC[e] = (j0 + jj < no) ? C[i * ldc + j0 + jj] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int nj = no - j0 < CJ ? no - j0 : CJ;
    for (long idx = (long)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (long)gridDim.x * blockDim.x) {
        double2 acc[CJ];
#pragma unroll
        for (int jj = 0; jj < CJ; jj++) acc[jj] = make_double2(0.0, 0.0);
        for (int i = 0; i < nv; i++) {
            const double2 v = V[(long)i * ldv + idx];
#pragma unroll
            for (int jj = 0; jj < CJ; jj++) {
                const double2 c = sC[i * CJ + jj];
                acc[jj].x = fma(v.x, c.x, fma(-v.y, c.y, acc[jj].x));
                acc[jj].y = fma(v.x, c.y, fma(v.y, c.x, acc[jj].y));
            }
        }
#pragma unroll
        for (int jj = 0; jj < CJ; jj++)
            if (jj < nj) {
                double2 *o = O + (long)(j0 + jj) * ldo + idx;
                if (beta != 0.0) {
                    const double2 old = *o;
                    acc[jj].x += beta * old.x;
                    acc[jj].y += beta * old.y;
                }
                *o = acc[jj];
            }
    }
}

hipError_t launch_combine(const double2 *V, long ldv, int nv, const double2 *C_dev, int ldc, double2 *O, long ldo,
                          int no, long n, hipStream_t s, double beta) {
    if (nv > 128) return hipErrorInvalidValue;
    const int gx = 1024;
    if (no <= 8)
        hipLaunchKernelGGL(k_combine<8>, dim3(gx, 1), dim3(256), 0, s, V, ldv, nv, C_dev, ldc, O, ldo, no, n, beta);
    else if (no <= 16)
        hipLaunchKernelGGL(k_combine<16>, dim3(gx, 1), dim3(256), 0, s, V, ldv, nv, C_dev, ldc, O, ldo, no, n, beta);
    else
        hipLaunchKernelGGL(k_combine<24>, dim3(gx, (no + 23) / 24), dim3(256), 0, s, V, ldv, nv, C_dev, ldc, O, ldo,
                           no, n, beta);
    return hipGetLastError();
}

// y = a x + b y + c z over n reals (z may be null when c == 0)
template <class R>
__global__ void k_lincomb(long n, R a, const R *__restrict__ x, R b, R *__restrict__ y, R c, const R *__restrict__ z) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        R v = a * x[i] + b * y[i];
        if (z) v += c * z[i];
        y[i] = v;
    }
}

hipError_t launch_lincomb64(long nreal, double a, const double *x, double b, double *y, double c, const double *z,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_lincomb<double>, dim3(2048), dim3(256), 0, s, nreal, a, x, b, y, c, z);
    return hipGetLastError();
}
hipError_t launch_lincomb32(long nreal, float a, const float *x, float b, float *y, float c, const float *z,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_lincomb<float>, dim3(2048), dim3(256), 0, s, nreal, a, x, b, y, c, z);
    return hipGetLastError();
}

// FP64 native double2 [p][12][Vh][2]  <->  FP32 native float4 [p][6][Vh][2]
__global__ void k_convert(long nsite2, int Vh, int nvec, const double2 *__restrict__ d, float4 *__restrict__ f,
                          int to64, double2 *__restrict__ d_out, const float4 *__restrict__ f_in) {
    // one thread per (vector, parity, component pair, site-in-parity, copy)
    const long total = (long)nvec * 2 * 6 * Vh * 2;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        long r = e;
        const int c = r & 1;
        r >>= 1;
        const long h = r % Vh;
        r /= Vh;
        const int k2 = r % 6;
        r /= 6;
        const int p = r % 2;
        const long v = r / 2;
        const long base64 = v * nsite2 * 12;
        const long i0 = base64 + (((long)(p * 12 + 2 * k2) * Vh + h) * 2 + c);
        const long i1 = base64 + (((long)(p * 12 + 2 * k2 + 1) * Vh + h) * 2 + c);
        const long i32 = v * nsite2 * 6 + (((long)(p * 6 + k2) * Vh + h) * 2 + c);
        if (!to64) {
            const double2 a = d[i0], b = d[i1];
            f[i32] = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
        } else {
            const float4 q = f_in[i32];
            d_out[i0] = make_double2(q.x, q.y);
            d_out[i1] = make_double2(q.z, q.w);
        }
    }
}

hipError_t launch_to_f32(const Geo &g, int nvec, const double2 *src, float4 *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_convert, dim3(4096), dim3(256), 0, s, 4L * g.Vh, g.Vh, nvec, src, dst, 0, nullptr,
                       nullptr);
    return hipGetLastError();
}
// the same conversion for one even vector (the parity-0 block alone):
// FP64 double2 [12][Vh][2] <-> FP32 float4 [6][Vh][2]
__global__ void k_convert_even(int Vh, const double2 *__restrict__ d, float4 *__restrict__ f, int to64,
                               double2 *__restrict__ d_out, const float4 *__restrict__ f_in) {
    const long total = 6L * Vh * 2;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
        const int c = e & 1;
        const long r = e >> 1;
        const long h = r % Vh;
        const int k2 = (int)(r / Vh);
        const long i0 = ((long)(2 * k2) * Vh + h) * 2 + c;
        const long i1 = ((long)(2 * k2 + 1) * Vh + h) * 2 + c;
        const long i32 = ((long)k2 * Vh + h) * 2 + c;
        if (!to64) {
            const double2 a = d[i0], b = d[i1];
            f[i32] = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
        } else {
            const float4 q = f_in[i32];
            d_out[i0] = make_double2(q.x, q.y);
            d_out[i1] = make_double2(q.z, q.w);
        }
    }
}

hipError_t launch_even_to_f32(const Geo &g, const double2 *src, float4 *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_convert_even, dim3(2048), dim3(256), 0, s, g.Vh, src, dst, 0, nullptr, nullptr);
    return hipGetLastError();
}
hipError_t launch_even_to_f64(const Geo &g, const float4 *src, double2 *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_convert_even, dim3(2048), dim3(256), 0, s, g.Vh, nullptr, nullptr, 1, dst, src);
    return hipGetLastError();
}

hipError_t launch_to_f64(const Geo &g, int nvec, const float4 *src, double2 *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_convert, dim3(4096), dim3(256), 0, s, 4L * g.Vh, g.Vh, nvec, nullptr, nullptr, 1, dst, src);
    return hipGetLastError();
}

// Gaussian complex entries from a counter-based hash (splitmix64 finaliser) + Box-Muller.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
    z += 0x9e3779b97f4a7c15ull;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
__global__ void k_gauss(double2 *__restrict__ x, long n, unsigned long long seed) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        const unsigned long long a = mix64(seed ^ mix64(2 * (unsigned long long)i));
        const unsigned long long b = mix64(seed ^ mix64(2 * (unsigned long long)i + 1));
        const double u1 = ((a >> 11) + 1.0) * (1.0 / 9007199254740993.0);
        const double u2 = (b >> 11) * (1.0 / 9007199254740992.0);
        const double r = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincospi(2.0 * u2, &sn, &cs);
        x[i] = make_double2(r * cs, r * sn);
    }
}
hipError_t launch_gauss(double2 *x, long n, unsigned long long seed, hipStream_t s) {
    hipLaunchKernelGGL(k_gauss, dim3(2048), dim3(256), 0, s, x, n, seed);
    return hipGetLastError();
}

}  // namespace cstar
