// Operator entry points (operator.hip).
#pragma once

#include "internal.hpp"

namespace lspr {

// Column blocking for ncol real columns per operator and products in precision prec
// (LSPR_FP32 or LSPR_FP64); the matrix-core kernel is used when the geometry holds tiles of
// that precision.
Cols make_cols(const Geometry& g, int ncol, int prec);
// Expansion terms per box and column for order P (after folding).
int expansion_terms(int P);

}  // namespace lspr
