// Internal entry of the preconditioner network used by the eigensolver (nn.cpp).
#pragma once

#include "cstar_internal.h"

namespace cstar {

// x_j <- M(x_j), j < nvec, for FP32 native spinors on the handle's stream with
// the network attached to the handle (ESTATE if none)
cstar_status nn_apply_block(cstar_gauge *g, float4 *xs, int nvec);

}  // namespace cstar
