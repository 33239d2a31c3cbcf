// Event-based kernel profiling (profile.cpp).
#pragma once

#include "internal.hpp"

namespace lspr {
namespace prof {

bool enabled();
// Whether a scope of this name records (all of them, or only the far-field ones in mode 2).
bool records(const char* name);
// Records a start event on s; the matching stop() records the end and the work counts.
// width: wavelengths (complex columns) of the launch, 0 when not applicable.
int start(const char* name, hipStream_t s);
void stop(int token, hipStream_t s, double flops, double bytes, double items, int width);

// RAII helper: a no-op when profiling is off.
struct Scope {
    int token = -1;
    hipStream_t s;
    double flops, bytes, items;
    int width;
    Scope(const char* name, hipStream_t st, double f, double b, double n = 0.0, int w = 0)
        : s(st), flops(f), bytes(b), items(n), width(w) {
        if (enabled() && records(name)) token = start(name, s);
    }
    ~Scope() {
        if (token >= 0) stop(token, s, flops, bytes, items, width);
    }
};

}  // namespace prof
}  // namespace lspr
