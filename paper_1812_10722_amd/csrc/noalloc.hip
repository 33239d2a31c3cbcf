// lspr_apply_noalloc: the block matrix-vector product of lspr_apply for callers that cannot
// allocate device memory (code under stream capture, tight serving loops).  Every temporary of
// the product (permittivity ratios, the sorted copies of x and y, packed densities, raw layer
// sums, box moments and partial moments) lives in one file-scope device array of fixed size,
// reached through the address the runtime reports for it on each device; the call allocates
// nothing and launches the same kernels as lspr_apply, in the same order, so its results are
// the same bit for bit.
#include <algorithm>
#include <map>
#include <mutex>
#include <string>

#include "driver.hpp"
#include "operator.hpp"
#include "system.hpp"

constexpr size_t SCRATCH_BYTES = static_cast<size_t>(LSPR_NOALLOC_SCRATCH_MIB) << 20;

// One copy per device, held from the library's load until the process ends.
static __device__ __align__(256) uint8_t scratch[SCRATCH_BYTES];

namespace {

// The device address of `scratch` on the current device (the array's name is a host-side
// stand-in in host code): looked up once per device and kept.
uint8_t* scratch_on_device() {
    static std::mutex mu;
    static std::map<int, uint8_t*> addr;
    int dev = 0;
    LSPR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) return it->second;
    void* p = nullptr;
    LSPR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    LSPR_REQUIRE(p != nullptr, LSPR_E_DEVICE, "no device address for the scratch array");
    addr[dev] = static_cast<uint8_t*>(p);
    return static_cast<uint8_t*>(p);
}

}  // namespace

namespace lspr {

size_t apply_scratch_bytes(const Geometry& g, int B, int prec) {
    const Cols c = make_cols(g, 2 * B, prec);
    const size_t esz = c.prec == LSPR_FP32 ? 4 : 8;
    const size_t nvec = 2 * static_cast<size_t>(g.N);
    const size_t nd = static_cast<size_t>(g.N) * 2 * c.pad;
    size_t b = arena_piece(static_cast<size_t>(B) * g.S * sizeof(double2));  // ratios
    b += 2 * arena_piece(static_cast<size_t>(B) * nvec * sizeof(double2));   // x, y sorted
    b += arena_piece(nd * esz);                                              // densities
    b += arena_piece(nd * sizeof(double) * (g.S > 1 ? 2 : 1));               // raw sums
    if (!g.mom_boxes.empty()) {
        b += arena_piece(g.mom_boxes.size() * g.n_terms * 2 * c.pad * esz);  // moments
        if (g.n_slots > 0)
            b += arena_piece(static_cast<size_t>(g.n_slots) * g.n_terms * 2 * c.pad * esz);
    }
    if (c.mfma && far_part_bytes(g, c.pad) > 0)                          // far-field pieces
        b += arena_piece(far_part_bytes(g, c.pad));
    return b;
}

}  // namespace lspr

extern "C" int lspr_apply_noalloc(lspr_geometry* h, int32_t n_cols, const lspr_c64* eps_medium,
                                  const lspr_c64* eps_surface, const lspr_c64* x, lspr_c64* y,
                                  void* stream) {
    return lspr::guarded([&] {
        LSPR_REQUIRE(h && eps_medium && eps_surface && x && y && n_cols >= 1, LSPR_E_INVALID,
                     "bad arguments");
        lspr::Geometry& g = h->g;
        hipStream_t s = static_cast<hipStream_t>(stream);
        const int prec = g.need64 ? LSPR_FP64 : LSPR_FP32;  // as lspr_apply
        const int B0 = std::min(lspr::MAX_BATCH, static_cast<int>(n_cols));
        const size_t need = lspr::apply_scratch_bytes(g, B0, prec);
        LSPR_REQUIRE(need <= SCRATCH_BYTES, LSPR_E_INVALID,
                     "lspr_apply_noalloc: this product needs " + std::to_string(need) +
                         " bytes of scratch, more than the library's fixed " +
                         std::to_string(SCRATCH_BYTES) + " (use lspr_apply, or fewer columns)");
        uint8_t* base = scratch_on_device();
        const int64_t nvec = 2 * static_cast<int64_t>(g.N);
        lspr::Geometry::Arena arena;
        arena.base = base;
        arena.cap = SCRATCH_BYTES;
        struct Restore {  // the geometry takes its own workspaces again afterwards
            lspr::Geometry& g;
            ~Restore() { g.arena = nullptr; }
        } restore{g};
        for (int b0 = 0; b0 < n_cols; b0 += lspr::MAX_BATCH) {
            const int B = std::min(lspr::MAX_BATCH, n_cols - b0);
            lspr::EpsSet e;
            for (int b = 0; b < B; ++b) {
                e.em_re.push_back(eps_medium[b0 + b].re);
                e.em_im.push_back(eps_medium[b0 + b].im);
                for (int k = 0; k < g.S; ++k) {
                    e.es_re.push_back(eps_surface[(b0 + b) * g.S + k].re);
                    e.es_im.push_back(eps_surface[(b0 + b) * g.S + k].im);
                }
            }
            const std::vector<double2> rh = lspr::ratio_values(g, e, B);
            arena.used = 0;
            g.arena = &arena;
            // the same pieces, in the same order, as apply_scratch_bytes counts
            auto piece = [&](size_t bytes) {
                return reinterpret_cast<double2*>(lspr::workspace(g, g.ws_dens, bytes));
            };
            double2* ratio = piece(rh.size() * sizeof(double2));
            double2* xs = piece(B * nvec * sizeof(double2));
            double2* ys = piece(B * nvec * sizeof(double2));
            LSPR_HIP(hipMemcpyAsync(ratio, rh.data(), rh.size() * sizeof(double2),
                                    hipMemcpyHostToDevice, s));
            lspr::to_sorted(g, B, reinterpret_cast<const double2*>(x) + b0 * nvec, xs, s);
            lspr::system_apply(g, prec, B, ratio, xs, nvec, ys, nvec, nullptr, s);
            lspr::from_sorted(g, B, ys, reinterpret_cast<double2*>(y) + b0 * nvec, s);
            g.arena = nullptr;
            LSPR_HIP(hipStreamSynchronize(s));  // rh is local; the next batch reuses the array
        }
        return static_cast<int>(LSPR_OK);
    });
}
