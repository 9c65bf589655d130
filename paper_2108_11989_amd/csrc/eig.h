// Eigensolver and sign-driver internals of libcstar.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/cstar.h"

namespace cstar {

// Optional preconditioner replacing the Chebyshev filter: Y = T(X) for nb FP64 vectors.
struct EigHooks {
    void *ctx;
    cstar_status (*precondition)(void *ctx, cstar_gauge *g, double m0, const double2 *X, int nb, double2 *Y);
};

cstar_status eig_lowest(cstar_gauge *g, double m0, int k, const cstar_eig_opts *opts, double *evals, double *resid,
                        void *evecs, cstar_eig_stats *stats, const EigHooks *hooks);
void workspace_release(cstar_gauge *g);

}  // namespace cstar
