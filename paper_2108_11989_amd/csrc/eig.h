// Eigensolver and sign-driver internals of libcstar.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/cstar.h"

namespace cstar {

// k lowest |lambda| of Q(m0), one per Kramers pair (q_lowest_eigs without the
// fallback).  opts->use_nn with a network attached to g: every iteration
// appends the preconditioned residuals M r_j of the wanted Ritz pairs to the
// filtered block.
cstar_status eig_lowest(cstar_gauge *g, double m0, int k, const cstar_eig_opts *opts, double *evals, double *resid,
                        void *evecs, cstar_eig_stats *stats);
void workspace_release(cstar_gauge *g);

}  // namespace cstar
