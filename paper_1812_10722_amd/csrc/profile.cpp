// Event-based kernel profiling: HIP events recorded on the launch stream around a launch, plus
// the algorithmic flops and bytes of that launch.  Events are kept until the next reset.
#include "profile.hpp"

#include <climits>
#include <cstring>
#include <map>
#include <mutex>

namespace lspr {
namespace prof {

namespace {

struct Rec {
    std::string name;
    hipEvent_t a = nullptr, b = nullptr;
    int dev = 0;
    double flops = 0, bytes = 0, items = 0;
    int width = 0;
    bool done = false;
};

std::mutex mu;
bool on = false;
int mode = 0;  // 1: every scope, 2: far-field scopes only
std::vector<Rec> recs;
// events of earlier records, per device, reused (creating one costs microseconds)
std::map<int, std::vector<hipEvent_t>> spare;

hipEvent_t take_event(int dev) {
    std::vector<hipEvent_t>& pool = spare[dev];
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    LSPR_HIP(hipEventCreate(&e));
    return e;
}

void clear_locked() {
    for (Rec& r : recs) {
        if (r.a) spare[r.dev].push_back(r.a);
        if (r.b) spare[r.dev].push_back(r.b);
    }
    recs.clear();
}

}  // namespace

bool enabled() { return on; }

bool records(const char* name) {
    return mode != 2 || std::strcmp(name, "far") == 0 || std::strcmp(name, "far64") == 0;
}

int start(const char* name, hipStream_t s) {
    std::lock_guard<std::mutex> lk(mu);
    Rec r;
    r.name = name;
    LSPR_HIP(hipGetDevice(&r.dev));
    r.a = take_event(r.dev);
    r.b = take_event(r.dev);
    LSPR_HIP(hipEventRecord(r.a, s));
    recs.push_back(r);
    return static_cast<int>(recs.size()) - 1;
}

void stop(int token, hipStream_t s, double flops, double bytes, double items, int width) {
    std::lock_guard<std::mutex> lk(mu);
    if (token < 0 || token >= static_cast<int>(recs.size())) return;
    Rec& r = recs[token];
    (void)hipEventRecord(r.b, s);
    r.flops = flops;
    r.bytes = bytes;
    r.items = items;
    r.width = width;
    r.done = true;
}

}  // namespace prof
}  // namespace lspr

extern "C" {

int lspr_profile_enable(int32_t enable) {
    if (enable < 0 || enable > 2) return LSPR_E_INVALID;
    lspr::prof::on = enable != 0;
    lspr::prof::mode = enable;
    return LSPR_OK;
}

int lspr_profile_reset(void) {
    std::lock_guard<std::mutex> lk(lspr::prof::mu);
    lspr::prof::clear_locked();
    return LSPR_OK;
}

int lspr_profile_query(const char* name, double* total_ms, int64_t* launches, double* flops,
                       double* bytes, double* items) {
    return lspr_profile_query_width(name, 0, INT32_MAX, total_ms, launches, flops, bytes, items);
}

int lspr_profile_query_width(const char* name, int32_t width_min, int32_t width_max,
                             double* total_ms, int64_t* launches, double* flops, double* bytes,
                             double* items) {
    if (!name || !total_ms || !launches || !flops || !bytes || !items) return LSPR_E_INVALID;
    std::lock_guard<std::mutex> lk(lspr::prof::mu);
    double ms = 0, f = 0, by = 0, it = 0;
    int64_t n = 0;
    for (auto& r : lspr::prof::recs) {
        if (!r.done || r.name != name || r.width < width_min || r.width > width_max) continue;
        if (hipEventSynchronize(r.b) != hipSuccess) return LSPR_E_DEVICE;
        float t = 0.f;
        if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return LSPR_E_DEVICE;
        ms += t;
        f += r.flops;
        by += r.bytes;
        it += r.items;
        ++n;
    }
    *total_ms = ms;
    *launches = n;
    *flops = f;
    *bytes = by;
    *items = it;
    return LSPR_OK;
}

}  // extern "C"
