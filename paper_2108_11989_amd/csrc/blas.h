// Launchers of the vector kernels (kernels_blas.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace cstar {
struct Geo;

int gram_blocks();
size_t gram_partial_bytes();
// G (device, nv x nw row-major complex) = V^H W over n complex entries; nv, nw <= 64
hipError_t launch_gram(const double2 *V, long ldv, int nv, const double2 *W, long ldw, int nw, long n,
                       double2 *partial, double2 *out_dev, hipStream_t s);
// O_j = beta O_j + sum_i V_i C[i*ldc + j], nv <= 128, O must not alias V
hipError_t launch_combine(const double2 *V, long ldv, int nv, const double2 *C_dev, int ldc, double2 *O, long ldo,
                          int no, long n, hipStream_t s, double beta = 0.0);
// x^H y of two FP32 native vectors of n4 float4 (FP64 accumulation) into out_dev
hipError_t launch_dot32(const float4 *x, const float4 *y, long n4, double2 *partial, double2 *out_dev,
                        hipStream_t s);
hipError_t launch_lincomb64(long nreal, double a, const double *x, double b, double *y, double c, const double *z,
                            hipStream_t s);
hipError_t launch_lincomb32(long nreal, float a, const float *x, float b, float *y, float c, const float *z,
                            hipStream_t s);
hipError_t launch_to_f32(const Geo &g, int nvec, const double2 *src, float4 *dst, hipStream_t s);
hipError_t launch_to_f64(const Geo &g, int nvec, const float4 *src, double2 *dst, hipStream_t s);
// one even vector (parity-0 block) FP64 <-> FP32 native
hipError_t launch_even_to_f32(const Geo &g, const double2 *src, float4 *dst, hipStream_t s);
hipError_t launch_even_to_f64(const Geo &g, const float4 *src, double2 *dst, hipStream_t s);
hipError_t launch_gauss(double2 *x, long n, unsigned long long seed, hipStream_t s);
}  // namespace cstar
