// Operator entry points (operator.hip).
#pragma once

#include "internal.hpp"

namespace lspr {

// Column blocking for ncol real columns per operator.
Cols make_cols(int ncol);
// Expansion terms per box and column for order P (after folding).
int expansion_terms(int P);

}  // namespace lspr
