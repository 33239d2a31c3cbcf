// Event-based kernel profiling (profile.cpp).
#pragma once

#include "internal.hpp"

namespace lspr {
namespace prof {

bool enabled();
// Records a start event on s; the matching stop() records the end and the work counts.
int start(const char* name, hipStream_t s);
void stop(int token, hipStream_t s, double flops, double bytes, double items);

// RAII helper: a no-op when profiling is off.
struct Scope {
    int token = -1;
    hipStream_t s;
    double flops, bytes, items;
    Scope(const char* name, hipStream_t st, double f, double b, double n = 0.0)
        : s(st), flops(f), bytes(b), items(n) {
        if (enabled()) token = start(name, s);
    }
    ~Scope() {
        if (token >= 0) stop(token, s, flops, bytes, items);
    }
};

}  // namespace prof
}  // namespace lspr
