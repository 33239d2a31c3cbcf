// Device primitives (primitives.hip).
#pragma once

#include "internal.hpp"

namespace lspr {

// out[i] = sum_{k<i} in[k] for i < n, out[n] = total.  out needs n + 1 entries; may alias in.
void scan_exclusive(const int64_t* in, int64_t* out, int64_t n, hipStream_t s);

// Stable ascending sort of (key, value) pairs on the low key_bits bits of the keys.
// Synchronises the stream before returning.
void radix_sort_pairs(uint64_t* keys, int32_t* vals, int64_t n, int key_bits, hipStream_t s);

}  // namespace lspr
