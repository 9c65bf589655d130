// Launchers of the preconditioner-network kernels (kernels_nn.hip).
#pragma once

#include "cstar_internal.h"

namespace cstar {

// out (cout channels) = layer(W) applied to in (cin channels); FP32 native
// spinor blocks with one spinor (24 Vh float4) per channel.  cin, cout in {1, 8}.
hipError_t launch_nn_layer(const Geo &g, const GaugeDev &d, const float4 *in, int cin, float4 *out, int cout,
                           const float *W, hipStream_t s);
// grad (FP64, [cout][cin][9][16] complex) += weight gradient of a layer with
// input `in` and output gradient `gout`; partial: nn_wgrad_blocks * cout*cin*9*32 doubles
int nn_wgrad_blocks(const Geo &g);
hipError_t launch_nn_wgrad(const Geo &g, const GaugeDev &d, const float4 *in, int cin, const float4 *gout, int cout,
                           double *partial, double *grad, hipStream_t s);
// Wt = weights of the input-gradient pass of a (cout x cin) layer
hipError_t launch_nn_wt(const float *W, int cout, int cin, float *Wt, hipStream_t s);
// gout = scale (y - x) (gout may be null), partial[nn_resid_blocks] = |y - x|^2 per block
int nn_resid_blocks();
hipError_t launch_nn_resid(long n4, const float4 *y, const float4 *x, float scale, float4 *gout, double *partial,
                           hipStream_t s);
hipError_t launch_nn_adam(int n, float *w, const double *grad, float *m, float *v, float b1, float b2, float step,
                          float eps_hat, hipStream_t s);

}  // namespace cstar
