// Eigensolver and sign-driver internals of libcstar.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/cstar.h"

namespace cstar {

// opts->use_nn with a network attached to g: the Chebyshev filter acts on M X
cstar_status eig_lowest(cstar_gauge *g, double m0, int k, const cstar_eig_opts *opts, double *evals, double *resid,
                        void *evecs, cstar_eig_stats *stats);
void workspace_release(cstar_gauge *g);

}  // namespace cstar
