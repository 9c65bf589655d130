// Internal declarations shared by the HIP kernels and the host code of libcstar.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <string>

#include "../../include/cstar.h"

namespace cstar {

// Geometry of the x-doubled C* lattice in the pair representation: every
// physical site (t,x1,x2,x3) carries two components, mirror 0 (the site
// itself) and mirror 1 (its charge-conjugate copy at x1+L).  Pairs are
// ordered even/odd: parity p = (t+x1+x2+x3)&1, in-parity index
// h = lex/2 with lex = ((t*L+x1)*L+x2)*L+x3.
struct Geo {
    int T, L, Lh;  // Lh = L/2
    int Vh;        // pairs per parity = T*L^3/2
    int time_bc;   // +1 / -1
};

// ---- device buffers owned by one handle ----------------------------------
struct GaugeDev {
    // FP64 quark links V = exp(i q theta) U: double2 [p][mu][9][Vh]
    double2 *link64 = nullptr;
    // FP32 rows 0,1 of U: float4 [p][mu][3][Vh]; BF16 rows 0,1: uint4 [p][mu][Vh] + uint2 [p][mu][Vh]
    float4 *link32 = nullptr;
    uint4 *linkbf_a = nullptr;
    uint2 *linkbf_b = nullptr;
    // quark phase exp(i q theta) as FP32 (cos, sin): float2 [p][mu][Vh]
    float2 *phase32 = nullptr;
    // clover, two Hermitian 6x6 blocks (36 reals each): FP64 double2 [p][36][Vh], FP32 float4 [p][18][Vh]
    double2 *clov64 = nullptr;
    float4 *clov32 = nullptr;
};

struct Workspace;  // eigensolver scratch (eig.cpp)

}  // namespace cstar

struct cstar_gauge {
    cstar_params par;
    cstar::Geo geo;
    int device = 0;
    hipStream_t stream = nullptr;
    cstar::GaugeDev d;
    double clover_norm_max = -1.0;
    cstar::Workspace *ws = nullptr;
    void *nn = nullptr;     // learned preconditioner state (nn.cpp), nullptr = none
    void *extra = nullptr;  // per-handle staging buffers (api.cpp)
    void *timing = nullptr; // apply-kernel event timing (timing.cpp), nullptr = off
    void *eo = nullptr;     // even-odd state (eo.cpp): inverse blocks of the last mass, scratch
};

namespace cstar {

void set_error(const std::string &msg);
cstar_status fail(cstar_status st, const std::string &msg);
#define CSTAR_HIP(call)                                                                        \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return ::cstar::fail(CSTAR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---- kernel launchers (kernels_dirac.hip) ---------------------------------
hipError_t launch_pack_links(const Geo &g, const double *su3, const double *theta, double q, GaugeDev &d,
                             hipStream_t s);
hipError_t launch_clover(const Geo &g, const double *su3, const double *theta, double q, double csw_su3,
                         double csw_u1, GaugeDev &d, double *norm_partial, hipStream_t s);
int clover_norm_blocks(const Geo &g);

// out_j = a_j * [g5] D(m_j) in_j  for j < nrhs; spinors native; strides in elements of the vector type
struct ApplyArgs {
    const void *in;
    void *out;
    long stride;      // distance between right-hand sides, in bytes
    int nrhs;
    int gamma5;
    const double *masses_dev;  // device [nrhs] (nullptr: use mass0)
    double mass0;
    // optional epilogue: out = ea * ([g5] D in) + eb * y + ec * z + ew[j] * w  (each of y, z, w optional,
    // same layout and stride; ew: device coefficients per right-hand side, float for the FP32 forms,
    // double for FP64)
    const void *y = nullptr;
    const void *z = nullptr;
    double ea = 1.0, eb = 0.0, ec = 0.0;
    const void *w = nullptr;
    const void *ew = nullptr;
    // with gamma5: Q + shift = g5 (D + shift g5), a spin-dependent local mass
    double shift = 0.0;
    // 1: never measure schedules (callers that must not synchronise or create
    // events): a cached choice or the default schedule
    int no_tune = 0;
};
hipError_t launch_apply(const Geo &g, const GaugeDev &d, cstar_prec prec, const ApplyArgs &a, hipStream_t s);
// Schedule of a multi-RHS time-marching launch (tune.cpp): the fastest of the
// kMarchSchedules candidates for this (precision, lattice, nrhs, epilogue),
// measured with HIP events on the first such launch, or read from the cache
// file named by CSTAR_TUNE_CACHE; CSTAR_MARCH_SCHEDULE forces one.  launch(s)
// issues the whole apply with schedule s (every schedule gives the same result).
constexpr int kMarchSchedules = 13;
int march_schedule(const Geo &g, cstar_prec prec, const ApplyArgs &a, hipStream_t s,
                   const std::function<void(int)> &launch);
// launch_apply on the handle's stream, with event timing when enabled (timing.cpp)
hipError_t handle_apply(cstar_gauge *g, cstar_prec prec, const ApplyArgs &a);
void timing_release(cstar_gauge *g);

hipError_t launch_pack_spinor(const Geo &g, cstar_prec prec, int nrhs, void *canon, void *native, int unpack,
                              hipStream_t s);

// ---- even-odd decomposition (kernels_eo.hip) ------------------------------
// D_hat psi_e on nrhs right-hand sides: in / out are parity-0 blocks (the first
// half of a native vector, stride_in / stride_out bytes apart), tmp full native
// vectors whose parity-1 blocks receive D_oo^{-1} D_oe psi_e; inv the inverse
// blocks of (4+m) + SW on the odd sites (FP64 double2 [36][Vh], FP32 float4 [18][Vh]).
struct EoArgs {
    const void *in;
    void *tmp;
    void *out;
    long stride_in, stride_tmp, stride_out;  // bytes
    int nrhs;
    double m;
    int gamma5;
    const void *inv;
};
int eo_pairs_blocks(const Geo &g);
hipError_t launch_local_inv(const Geo &g, const GaugeDev &d, double m, double2 *inv64, float4 *inv32, hipStream_t s);
hipError_t launch_logdet_ratio(const Geo &g, const GaugeDev &d, double m, double mp, double *partial, hipStream_t s);
hipError_t launch_eo_apply(const Geo &g, const GaugeDev &d, cstar_prec prec, const EoArgs &e, hipStream_t s);
void eo_release(cstar_gauge *g);
cstar_status sign_driver_stepa(cstar_lbar_provider lbar, cstar_eig_provider prov, void *ctx, const double *m_path,
                               int n, int k, double c, double m_max, int *sign_out, cstar_sign_report *report);
cstar_status eo_apply(cstar_gauge *g, int nrhs, double m0, cstar_prec prec, int gamma5, const void *in, void *out);
// y += a (g5)^k x on n FP64 even vectors (complex a; g5 when k = 1)
hipError_t launch_even_axpy(const Geo &g, double are, double aim, int g5, const void *x, void *y, hipStream_t s);

// ---- BLAS on native vectors (kernels_blas.hip) -----------------------------
// A native FP64 vector is an array of n2 = 24*Vh*... double2 entries (complex numbers);
// an FP32 vector is an array of n4 float4 entries (two complex numbers each).
long n_cplx(const Geo &g);  // complex entries per spinor = 2*T*L^3*12

}  // namespace cstar
