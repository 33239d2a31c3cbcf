// Operator entry points (operator.hip).
#pragma once

#include "internal.hpp"

namespace lspr {

// Column blocking for ncol real columns per operator; FP32 products with at least 16 columns
// use the matrix-core kernel unless allow_mfma is false.
Cols make_cols(int ncol, int precision, bool allow_mfma = true);
// Expansion terms per box and column for order P (after folding).
int expansion_terms(int P);

}  // namespace lspr
