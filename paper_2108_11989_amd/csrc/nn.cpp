// Gauge-covariant preconditioner network: device state, loss and gradient,
// Adam training and inference (C ABI in include/cstar.h, cstar_nn_*).
//
// The network is not part of the paper's method; it is an optional
// preconditioner of the eigensolver.  Three layers (channels 1 -> 8 -> 8 -> 1)
// of the parallel-transport convolution of kernels_nn.hip.  It is trained to
// approximate (Q^2)^-1 with the loss
//   L = (1/N) sum_i |M(b_i) - x_i|^2 / |x_i|^2,   b_i = Q(m)^2 x_i.
// Backward pass, for out = W u:  grad W = sum g_out (x) conj(u), and the
// input gradient of a layer is the layer with weights W[a][b][rev p]^H.
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "cstar_internal.h"
#include "nn.h"
#include "nn_kernels.h"

namespace cstar {

namespace {
constexpr int CH[4] = {1, 8, 8, 1};
constexpr long layer_floats(int l) { return (long)CH[l + 1] * CH[l] * 9 * 32; }
constexpr long layer_offset(int l) { return l == 0 ? 0 : layer_offset(l - 1) + layer_floats(l - 1); }
static_assert(layer_offset(3) == CSTAR_NN_PARAMS, "parameter count");

// activation channels (FP32 native spinors) of one forward + backward pass
enum { A_H1 = 0, A_H2 = 8, A_Y = 16, A_GY = 17, A_GH2 = 18, A_GH1 = 26, A_NCH = 34 };
}  // namespace

}  // namespace cstar

struct cstar_nn {
    int device = 0;
    float *w = nullptr;     // weights [CSTAR_NN_PARAMS]
    float *wt = nullptr;    // input-gradient weights (same offsets)
    float *m = nullptr, *v = nullptr;  // Adam moments
    double *grad = nullptr;            // accumulated gradient
    long steps = 0;                    // Adam steps taken
    // activations for one geometry
    int vh = 0;
    int nch = 0;
    float4 *act = nullptr;
    double *partial = nullptr;  // wgrad / residual partial sums
    size_t partial_n = 0;
};

namespace cstar {

namespace {

cstar_status ensure_act(cstar_nn *nn, const Geo &g, bool training) {
    const int need = training ? A_NCH : A_Y + 1;
    if (nn->act && nn->vh == g.Vh && nn->nch >= need) return CSTAR_OK;
    if (nn->act) (void)hipFree(nn->act);
    if (nn->partial) (void)hipFree(nn->partial);
    nn->act = nullptr;
    nn->partial = nullptr;
    const size_t cs = 24ul * g.Vh;
    size_t pn = (size_t)nn_wgrad_blocks(g) * 8 * 8 * 9 * 32;
    if (pn < (size_t)nn_resid_blocks()) pn = nn_resid_blocks();
    if (hipMalloc(&nn->act, sizeof(float4) * cs * need) != hipSuccess ||
        hipMalloc(&nn->partial, sizeof(double) * pn) != hipSuccess) {
        (void)hipGetLastError();
        if (nn->act) (void)hipFree(nn->act);
        nn->act = nullptr;
        nn->partial = nullptr;
        return fail(CSTAR_ENOMEM, "cstar_nn: device allocation of activations failed");
    }
    nn->vh = g.Vh;
    nn->nch = need;
    nn->partial_n = pn;
    return CSTAR_OK;
}

float4 *chan(cstar_nn *nn, int c) { return nn->act + 24L * nn->vh * c; }

// y = M(b) for one vector; h1, h2 kept in the activation buffer
cstar_status forward(cstar_nn *nn, cstar_gauge *g, const float4 *b, float4 *y) {
    CSTAR_HIP(launch_nn_layer(g->geo, g->d, b, 1, chan(nn, A_H1), 8, nn->w + layer_offset(0), g->stream));
    CSTAR_HIP(launch_nn_layer(g->geo, g->d, chan(nn, A_H1), 8, chan(nn, A_H2), 8, nn->w + layer_offset(1), g->stream));
    CSTAR_HIP(launch_nn_layer(g->geo, g->d, chan(nn, A_H2), 8, y, 1, nn->w + layer_offset(2), g->stream));
    return CSTAR_OK;
}

// sum over blocks of a partial array, in order, on the host
cstar_status host_sum(cstar_gauge *g, const double *partial, int n, double *out) {
    std::vector<double> h(n);
    CSTAR_HIP(hipMemcpyAsync(h.data(), partial, sizeof(double) * n, hipMemcpyDeviceToHost, g->stream));
    CSTAR_HIP(hipStreamSynchronize(g->stream));
    double s = 0.0;
    for (double v : h) s += v;
    *out = s;
    return CSTAR_OK;
}

bool same_device(cstar_nn *nn, cstar_gauge *g) {
    int dev = -1;
    return hipGetDevice(&dev) == hipSuccess && dev == nn->device && g->device == nn->device;
}

}  // namespace

cstar_status nn_apply_block(cstar_gauge *g, float4 *xs, int nvec) {
    cstar_nn *nn = (cstar_nn *)g->nn;
    if (!nn) return fail(CSTAR_ESTATE, "no network attached");
    cstar_status st = ensure_act(nn, g->geo, false);
    if (st) return st;
    const long cs = 24L * g->geo.Vh;
    for (int j = 0; j < nvec; j++) {
        // in place: layer 0 consumes x_j before layer 2 writes it
        st = forward(nn, g, xs + j * cs, xs + j * cs);
        if (st) return st;
    }
    return CSTAR_OK;
}

namespace {

// loss contribution and gradient accumulation of the pairs (x_i, b_i), i < nvec
cstar_status loss_grad(cstar_nn *nn, cstar_gauge *g, int nvec, const float4 *x, const float4 *b, int n_total,
                       double *loss) {
    cstar_status st = ensure_act(nn, g->geo, true);
    if (st) return st;
    const Geo &geo = g->geo;
    const long cs = 24L * geo.Vh;
    CSTAR_HIP(launch_nn_wt(nn->w + layer_offset(1), 8, 8, nn->wt + layer_offset(1), g->stream));
    CSTAR_HIP(launch_nn_wt(nn->w + layer_offset(2), 1, 8, nn->wt + layer_offset(2), g->stream));
    double total = 0.0;
    for (int i = 0; i < nvec; i++) {
        const float4 *xi = x + i * cs, *bi = b + i * cs;
        double nx = 0.0;
        CSTAR_HIP(launch_nn_resid(cs, xi, nullptr, 0.f, nullptr, nn->partial, g->stream));
        st = host_sum(g, nn->partial, nn_resid_blocks(), &nx);
        if (st) return st;
        if (!(nx > 0.0)) return fail(CSTAR_EINVAL, "cstar_nn_loss_grad: zero target vector");
        st = forward(nn, g, bi, chan(nn, A_Y));
        if (st) return st;
        const double scale = 2.0 / (nx * n_total);
        CSTAR_HIP(launch_nn_resid(cs, chan(nn, A_Y), xi, (float)scale, chan(nn, A_GY), nn->partial, g->stream));
        double r2 = 0.0;
        st = host_sum(g, nn->partial, nn_resid_blocks(), &r2);
        if (st) return st;
        total += r2 / (nx * n_total);
        // layer 2: input h2, output gradient gy
        CSTAR_HIP(launch_nn_wgrad(geo, g->d, chan(nn, A_H2), 8, chan(nn, A_GY), 1, nn->partial,
                                  nn->grad + layer_offset(2), g->stream));
        CSTAR_HIP(launch_nn_layer(geo, g->d, chan(nn, A_GY), 1, chan(nn, A_GH2), 8, nn->wt + layer_offset(2), g->stream));
        // layer 1: input h1, output gradient gh2
        CSTAR_HIP(launch_nn_wgrad(geo, g->d, chan(nn, A_H1), 8, chan(nn, A_GH2), 8, nn->partial,
                                  nn->grad + layer_offset(1), g->stream));
        CSTAR_HIP(launch_nn_layer(geo, g->d, chan(nn, A_GH2), 8, chan(nn, A_GH1), 8, nn->wt + layer_offset(1), g->stream));
        // layer 0: input b, output gradient gh1
        CSTAR_HIP(launch_nn_wgrad(geo, g->d, bi, 1, chan(nn, A_GH1), 8, nn->partial, nn->grad + layer_offset(0),
                                  g->stream));
    }
    CSTAR_HIP(hipStreamSynchronize(g->stream));
    *loss = total;
    return CSTAR_OK;
}

cstar_status adam_step(cstar_nn *nn, hipStream_t s, double lr, double b1, double b2, double eps) {
    nn->steps += 1;
    const double c1 = 1.0 - std::pow(b1, (double)nn->steps), c2 = 1.0 - std::pow(b2, (double)nn->steps);
    const double step = lr * std::sqrt(c2) / c1, eps_hat = eps * std::sqrt(c2);
    CSTAR_HIP(launch_nn_adam(CSTAR_NN_PARAMS, nn->w, nn->grad, nn->m, nn->v, (float)b1, (float)b2, (float)step,
                             (float)eps_hat, s));
    CSTAR_HIP(hipMemsetAsync(nn->grad, 0, sizeof(double) * CSTAR_NN_PARAMS, s));
    return CSTAR_OK;
}

void nn_free(cstar_nn *nn) {
    void *ptrs[] = {nn->w, nn->wt, nn->m, nn->v, nn->grad, nn->act, nn->partial};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete nn;
}

}  // namespace

}  // namespace cstar

using namespace cstar;

extern "C" {

cstar_status cstar_nn_create(const float *weights, cstar_nn **out) {
    if (!out) return fail(CSTAR_EINVAL, "cstar_nn_create: null argument");
    *out = nullptr;
    std::vector<float> w(CSTAR_NN_PARAMS, 0.f);
    if (weights) {
        for (long i = 0; i < CSTAR_NN_PARAMS; i++) {
            if (!std::isfinite(weights[i])) return fail(CSTAR_EINVAL, "cstar_nn_create: non-finite weight");
            w[i] = weights[i];
        }
    } else {
        // identity: channel 0 carries the input through path 0 of every layer
        for (int l = 0; l < 3; l++)
            for (int s = 0; s < 4; s++) w[layer_offset(l) + (s * 4 + s) * 2] = 1.f;
    }
    cstar_nn *nn = new (std::nothrow) cstar_nn();
    if (!nn) return fail(CSTAR_ENOMEM, "host allocation failed");
    (void)hipGetDevice(&nn->device);
    const size_t nf = sizeof(float) * CSTAR_NN_PARAMS;
    bool ok = hipMalloc(&nn->w, nf) == hipSuccess && hipMalloc(&nn->wt, nf) == hipSuccess &&
              hipMalloc(&nn->m, nf) == hipSuccess && hipMalloc(&nn->v, nf) == hipSuccess &&
              hipMalloc(&nn->grad, sizeof(double) * CSTAR_NN_PARAMS) == hipSuccess;
    ok = ok && hipMemcpy(nn->w, w.data(), nf, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemset(nn->wt, 0, nf) == hipSuccess && hipMemset(nn->m, 0, nf) == hipSuccess &&
         hipMemset(nn->v, 0, nf) == hipSuccess &&
         hipMemset(nn->grad, 0, sizeof(double) * CSTAR_NN_PARAMS) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        nn_free(nn);
        return fail(CSTAR_ENOMEM, "cstar_nn_create: device allocation failed");
    }
    *out = nn;
    return CSTAR_OK;
}

void cstar_nn_destroy(cstar_nn *nn) {
    if (!nn) return;
    (void)hipDeviceSynchronize();
    nn_free(nn);
}

cstar_status cstar_nn_get_weights(cstar_nn *nn, float *out) {
    if (!nn || !out) return fail(CSTAR_EINVAL, "cstar_nn_get_weights: null argument");
    CSTAR_HIP(hipDeviceSynchronize());
    CSTAR_HIP(hipMemcpy(out, nn->w, sizeof(float) * CSTAR_NN_PARAMS, hipMemcpyDeviceToHost));
    return CSTAR_OK;
}

cstar_status cstar_nn_set_weights(cstar_nn *nn, const float *w) {
    if (!nn || !w) return fail(CSTAR_EINVAL, "cstar_nn_set_weights: null argument");
    for (long i = 0; i < CSTAR_NN_PARAMS; i++)
        if (!std::isfinite(w[i])) return fail(CSTAR_EINVAL, "cstar_nn_set_weights: non-finite weight");
    CSTAR_HIP(hipDeviceSynchronize());
    CSTAR_HIP(hipMemcpy(nn->w, w, sizeof(float) * CSTAR_NN_PARAMS, hipMemcpyHostToDevice));
    return CSTAR_OK;
}

cstar_status cstar_nn_get_grad(cstar_nn *nn, double *out) {
    if (!nn || !out) return fail(CSTAR_EINVAL, "cstar_nn_get_grad: null argument");
    CSTAR_HIP(hipDeviceSynchronize());
    CSTAR_HIP(hipMemcpy(out, nn->grad, sizeof(double) * CSTAR_NN_PARAMS, hipMemcpyDeviceToHost));
    return CSTAR_OK;
}

cstar_status cstar_nn_zero_grad(cstar_nn *nn) {
    if (!nn) return fail(CSTAR_EINVAL, "cstar_nn_zero_grad: null argument");
    CSTAR_HIP(hipMemset(nn->grad, 0, sizeof(double) * CSTAR_NN_PARAMS));
    return CSTAR_OK;
}

cstar_status cstar_nn_apply(cstar_nn *nn, cstar_gauge *g, int nvec, const void *b, void *y) {
    if (!nn || !g || !b || !y || nvec < 1) return fail(CSTAR_EINVAL, "cstar_nn_apply: bad argument");
    if (!same_device(nn, g)) return fail(CSTAR_EINVAL, "cstar_nn_apply: network and handle on different devices");
    cstar_status st = ensure_act(nn, g->geo, false);
    if (st) return st;
    const long cs = 24L * g->geo.Vh;
    const float4 *bi = (const float4 *)b;
    float4 *yi = (float4 *)y;
    const size_t bytes = sizeof(float4) * cs * nvec;
    if ((const char *)bi < (const char *)yi + bytes && (const char *)yi < (const char *)bi + bytes && bi != yi)
        return fail(CSTAR_EINVAL, "cstar_nn_apply: b and y overlap partially");
    for (int j = 0; j < nvec; j++) {
        st = forward(nn, g, bi + j * cs, yi + j * cs);
        if (st) return st;
    }
    return CSTAR_OK;
}

cstar_status cstar_nn_loss_grad(cstar_nn *nn, cstar_gauge *g, int nvec, const void *x, const void *b, int n_total,
                                double *loss) {
    if (!nn || !g || !x || !b || !loss || nvec < 1 || n_total < 1)
        return fail(CSTAR_EINVAL, "cstar_nn_loss_grad: bad argument");
    if (!same_device(nn, g)) return fail(CSTAR_EINVAL, "cstar_nn_loss_grad: network and handle on different devices");
    return loss_grad(nn, g, nvec, (const float4 *)x, (const float4 *)b, n_total, loss);
}

cstar_status cstar_nn_adam_step(cstar_nn *nn, double lr, double beta1, double beta2, double eps) {
    if (!nn || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(CSTAR_EINVAL, "cstar_nn_adam_step: bad argument");
    cstar_status st = adam_step(nn, nullptr, lr, beta1, beta2, eps);
    if (st) return st;
    CSTAR_HIP(hipStreamSynchronize(nullptr));
    return CSTAR_OK;
}

cstar_status cstar_nn_train(cstar_nn *nn, cstar_gauge *const *fields, int n_fields, const void *const *x, int nvec,
                            double m0, int epochs, double lr, double *loss_history) {
    if (!nn || !fields || !x || n_fields < 1 || nvec < 1 || epochs < 1 || !(lr > 0) || !std::isfinite(m0))
        return fail(CSTAR_EINVAL, "cstar_nn_train: bad argument");
    const Geo &g0 = fields[0]->geo;
    for (int f = 0; f < n_fields; f++) {
        if (!fields[f] || !x[f]) return fail(CSTAR_EINVAL, "cstar_nn_train: null field or vector block");
        const Geo &gf = fields[f]->geo;
        if (gf.T != g0.T || gf.L != g0.L) return fail(CSTAR_EINVAL, "cstar_nn_train: fields of different lattices");
        if (!same_device(nn, fields[f])) return fail(CSTAR_EINVAL, "cstar_nn_train: field on another device");
    }
    const long cs = 24L * g0.Vh;
    const size_t vbytes = sizeof(float4) * cs;
    // b_i = Q(m0)^2 x_i for every field, in FP32
    float4 *B = nullptr, *tmp = nullptr;
    if (hipMalloc(&B, vbytes * nvec * n_fields) != hipSuccess || hipMalloc(&tmp, vbytes * nvec) != hipSuccess) {
        (void)hipGetLastError();
        if (B) (void)hipFree(B);
        return fail(CSTAR_ENOMEM, "cstar_nn_train: device allocation failed");
    }
    cstar_status st = CSTAR_OK;
    for (int f = 0; f < n_fields && !st; f++) {
        cstar_gauge *g = fields[f];
        ApplyArgs a1{x[f], tmp, (long)vbytes, nvec, 1, nullptr, m0};
        ApplyArgs a2{tmp, B + f * nvec * cs, (long)vbytes, nvec, 1, nullptr, m0};
        hipError_t e = handle_apply(g, CSTAR_FP32, a1);
        if (e == hipSuccess) e = handle_apply(g, CSTAR_FP32, a2);
        if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
        if (e != hipSuccess) st = fail(CSTAR_EDEVICE, std::string("cstar_nn_train: ") + hipGetErrorString(e));
    }
    for (int ep = 0; ep < epochs && !st; ep++) {
        double sum = 0.0;
        for (int f = 0; f < n_fields && !st; f++) {
            cstar_gauge *g = fields[f];
            double L = 0.0;
            st = loss_grad(nn, g, nvec, (const float4 *)x[f], B + f * nvec * cs, nvec, &L);
            if (!st) st = adam_step(nn, g->stream, lr, 0.9, 0.999, 1e-8);
            if (!st && !std::isfinite(L)) st = fail(CSTAR_ENOCONV, "cstar_nn_train: loss is not finite");
            sum += L;
        }
        if (!st && loss_history) loss_history[ep] = sum / n_fields;
    }
    (void)hipDeviceSynchronize();
    (void)hipFree(B);
    (void)hipFree(tmp);
    return st;
}

cstar_status cstar_nn_attach(cstar_gauge *g, cstar_nn *nn) {
    if (!g) return fail(CSTAR_EINVAL, "cstar_nn_attach: null handle");
    if (nn && !same_device(nn, g)) return fail(CSTAR_EINVAL, "cstar_nn_attach: network on another device");
    g->nn = nn;
    return CSTAR_OK;
}

}  // extern "C"
