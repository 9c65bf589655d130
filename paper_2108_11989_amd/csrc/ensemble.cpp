// W_sgn over an ensemble of gauge fields and quark flavours (C ABI in include/cstar.h).
//
// Paper, sign-of-the-Pfaffian section and summary: the sign of the Pfaffian
// enters the path integral as a reweighting factor of every configuration;
// with several quark flavours (charges, masses) the factor is the product of
// the flavours' signs.  One GPU, configurations in turn: for every
// configuration and flavour a handle is created on the field with that
// flavour's charge, pfaffian_sign is called at the flavour's target mass, and
// the handle is destroyed.  A flavour equal to an earlier one of the same
// configuration (same charge and mass) has the same sign and is not solved
// again.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <string>

#include "cstar_internal.h"

using namespace cstar;

extern "C" cstar_status cstar_sign_ensemble(const cstar_params *base, int n_cfg, const double *const *su3,
                                            const double *const *theta, int src_on_device, int n_flv,
                                            const double *charges, const double *m_target,
                                            const cstar_sign_opts *opts, int *sign_out, int *product_out,
                                            double *seconds_out) {
    if (!base || !su3 || !theta || !charges || !m_target || !opts || !sign_out || !product_out || n_cfg < 1 ||
        n_flv < 1)
        return fail(CSTAR_EINVAL, "cstar_sign_ensemble: bad argument");
    for (int c = 0; c < n_cfg; c++)
        if (!su3[c] || !theta[c]) return fail(CSTAR_EINVAL, "cstar_sign_ensemble: null field pointer");
    for (int f = 0; f < n_flv; f++)
        if (!std::isfinite(charges[f]) || !std::isfinite(m_target[f]))
            return fail(CSTAR_EINVAL, "cstar_sign_ensemble: non-finite charge or mass");
    cstar_status worst = CSTAR_OK;
    for (int c = 0; c < n_cfg; c++) {
        const auto t0 = std::chrono::steady_clock::now();
        int prod = 1;
        for (int f = 0; f < n_flv; f++) {
            int dup = -1;
            for (int e = 0; e < f; e++)
                if (charges[e] == charges[f] && m_target[e] == m_target[f]) dup = e;
            int sg = 0;
            if (dup >= 0) {
                sg = sign_out[(long)c * n_flv + dup];
            } else {
                cstar_params p = *base;
                p.q = charges[f];
                cstar_gauge *g = nullptr;
                cstar_status st = cstar_gauge_create(&p, su3[c], theta[c], src_on_device, nullptr, &g);
                if (st != CSTAR_OK)
                    return fail(st, "cstar_sign_ensemble: configuration " + std::to_string(c) + ": " + cstar_last_error());
                double m = m_target[f];
                st = pfaffian_sign(g, &m, 1, opts, &sg, nullptr);
                std::string msg = st != CSTAR_OK ? std::string(cstar_last_error()) : std::string();
                cstar_gauge_destroy(g);
                if (st == CSTAR_EAMBIG) {
                    sg = 0;
                    worst = CSTAR_EAMBIG;
                } else if (st != CSTAR_OK) {
                    return fail(st, "cstar_sign_ensemble: configuration " + std::to_string(c) + ", flavour " +
                                        std::to_string(f) + ": " + msg);
                }
            }
            sign_out[(long)c * n_flv + f] = sg;
            prod *= sg;
        }
        product_out[c] = prod;
        if (seconds_out)
            seconds_out[c] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (worst == CSTAR_EAMBIG)
        return fail(CSTAR_EAMBIG, "cstar_sign_ensemble: a sign could not be decided (its entries and products are 0)");
    return CSTAR_OK;
}
