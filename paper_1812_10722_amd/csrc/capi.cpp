// C ABI of the library (declared in include/lspr.h): argument checks, error translation and
// orchestration of the set-up and solve steps.
#include <algorithm>
#include <mutex>
#include <map>
#include <cmath>
#include <complex>
#include <future>
#include <utility>

#include "driver.hpp"
#include "operator.hpp"
#include "profile.hpp"
#include "system.hpp"

namespace {

using lspr::guarded;
using lspr::MAX_BATCH;

lspr::EpsSet make_eps(int B, int S, const lspr_c64* em, const lspr_c64* es) {
    lspr::EpsSet e;
    for (int b = 0; b < B; ++b) {
        e.em_re.push_back(em[b].re);
        e.em_im.push_back(em[b].im);
        for (int k = 0; k < S; ++k) {
            e.es_re.push_back(es[b * S + k].re);
            e.es_im.push_back(es[b * S + k].im);
        }
    }
    return e;
}

}  // namespace

namespace lspr {

std::string& last_error() {
    thread_local std::string text;
    return text;
}

AllocCtx& alloc_ctx() {
    thread_local AllocCtx ctx;
    return ctx;
}

hipMemPool_t library_pool() {
    static std::mutex mu;
    static std::map<int, hipMemPool_t> pools;
    int dev = 0;
    LSPR_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto it = pools.find(dev);
    if (it != pools.end()) return it->second;
    hipMemPoolProps props{};
    props.allocType = hipMemAllocationTypePinned;
    props.handleTypes = hipMemHandleTypeNone;
    props.location.type = hipMemLocationTypeDevice;
    props.location.id = dev;
    hipMemPool_t pool = nullptr;
    LSPR_HIP(hipMemPoolCreate(&pool, &props));
    uint64_t keep = 64ull << 30;
    LSPR_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep));
    pools[dev] = pool;
    return pool;
}

namespace {
struct CachedBlock {
    hipMemPool_t pool;
    void* p;
    size_t bytes;
    hipEvent_t ready;
};
std::mutex cache_mu;
std::vector<CachedBlock> cache;  // every device's pools; blocks are few and large
// Cached blocks are kept up to this many bytes per pool; a block that does not fit evicts smaller
// ones (a large block is the one that costs most to map again: the 96 GB FP64 tile store of a
// 491k-panel mesh), and an allocation that does not fit flushes the cache.
constexpr size_t CACHE_CAP = 128ull << 30;
size_t cached_bytes(hipMemPool_t pool) {
    size_t t = 0;
    for (const CachedBlock& b : cache) t += b.pool == pool ? b.bytes : 0;
    return t;
}
}  // namespace

void* big_block_take(hipMemPool_t pool, size_t bytes, hipStream_t s, size_t* got) {
    std::lock_guard<std::mutex> lk(cache_mu);
    // the smallest block that holds the request and wastes at most a quarter of it
    int best = -1;
    for (size_t i = 0; i < cache.size(); ++i) {
        const CachedBlock& b = cache[i];
        if (b.pool != pool || b.bytes < bytes || b.bytes > bytes + bytes / 4) continue;
        if (best < 0 || b.bytes < cache[best].bytes) best = static_cast<int>(i);
    }
    if (best < 0) return nullptr;
    const CachedBlock b = cache[best];
    cache.erase(cache.begin() + best);
    LSPR_HIP(hipStreamWaitEvent(s, b.ready, 0));
    (void)hipEventDestroy(b.ready);
    *got = b.bytes;
    return b.p;
}

bool big_block_put(hipMemPool_t pool, void* p, size_t bytes, hipStream_t s) {
    std::lock_guard<std::mutex> lk(cache_mu);
    size_t have = cached_bytes(pool);
    if (have + bytes > CACHE_CAP) {
        // room from smaller blocks of the pool, smallest first, if they free enough
        size_t smaller = 0;
        for (const CachedBlock& b : cache)
            if (b.pool == pool && b.bytes < bytes) smaller += b.bytes;
        if (have - smaller + bytes > CACHE_CAP) return false;
        while (have + bytes > CACHE_CAP) {
            int k = -1;
            for (size_t i = 0; i < cache.size(); ++i)
                if (cache[i].pool == pool && cache[i].bytes < bytes &&
                    (k < 0 || cache[i].bytes < cache[k].bytes))
                    k = static_cast<int>(i);
            const CachedBlock d = cache[k];
            cache.erase(cache.begin() + k);
            (void)hipEventSynchronize(d.ready);  // its last use has finished
            (void)hipEventDestroy(d.ready);
            (void)hipFreeAsync(d.p, s);  // back to the pool, which keeps it for reuse
            have -= d.bytes;
        }
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return false;
    if (hipEventRecord(ev, s) != hipSuccess) {
        (void)hipEventDestroy(ev);
        return false;
    }
    cache.push_back({pool, p, bytes, ev});
    return true;
}

namespace {
std::mutex pinned_mu;
std::vector<lspr::PinnedBuf> pinned_free;  // staging buffers not in use
// Free buffers are kept up to this many bytes in all (the largest first); freeing pinned memory
// can wait for the whole device, so a buffer is freed only when the pool is over its cap, and
// outside the lock.
constexpr size_t PINNED_KEEP_BYTES = 1ull << 30;
}  // namespace

PinnedBuf pinned_take(size_t bytes) {
    {
        // the smallest free buffer that holds the request
        std::lock_guard<std::mutex> lk(pinned_mu);
        int best = -1;
        for (size_t i = 0; i < pinned_free.size(); ++i)
            if (pinned_free[i].cap >= bytes &&
                (best < 0 || pinned_free[i].cap < pinned_free[best].cap))
                best = static_cast<int>(i);
        if (best >= 0) {
            const PinnedBuf b = pinned_free[best];
            pinned_free.erase(pinned_free.begin() + best);
            return b;
        }
    }
    PinnedBuf b;
    b.cap = ((bytes > 0 ? bytes : 1) + (1u << 20) - 1) & ~static_cast<size_t>((1u << 20) - 1);
    LSPR_HIP(hipHostMalloc(reinterpret_cast<void**>(&b.p), b.cap, hipHostMallocPortable));
    return b;
}

void pinned_put(PinnedBuf b) {
    if (b.p == nullptr) return;
    std::vector<PinnedBuf> drop;
    {
        std::lock_guard<std::mutex> lk(pinned_mu);
        pinned_free.push_back(b);
        size_t total = 0;
        for (const PinnedBuf& f : pinned_free) total += f.cap;
        while (total > PINNED_KEEP_BYTES && pinned_free.size() > 1) {  // drop the smallest
            size_t k = 0;
            for (size_t i = 1; i < pinned_free.size(); ++i)
                if (pinned_free[i].cap < pinned_free[k].cap) k = i;
            total -= pinned_free[k].cap;
            drop.push_back(pinned_free[k]);
            pinned_free.erase(pinned_free.begin() + k);
        }
    }
    for (const PinnedBuf& f : drop) (void)hipHostFree(f.p);
}

size_t reusable_bytes(hipMemPool_t pool) {
    if (pool == nullptr) return 0;
    size_t cached = 0;
    {
        std::lock_guard<std::mutex> lk(cache_mu);
        cached = cached_bytes(pool);
    }
    uint64_t reserved = 0, used = 0;
    if (hipMemPoolGetAttribute(pool, hipMemPoolAttrReservedMemCurrent, &reserved) != hipSuccess ||
        hipMemPoolGetAttribute(pool, hipMemPoolAttrUsedMemCurrent, &used) != hipSuccess)
        return cached;
    return cached + (reserved > used ? static_cast<size_t>(reserved - used) : 0);
}

bool big_block_flush(hipMemPool_t pool) {
    std::lock_guard<std::mutex> lk(cache_mu);
    bool any = false;
    for (size_t i = 0; i < cache.size();) {
        if (cache[i].pool != pool) {
            ++i;
            continue;
        }
        (void)hipEventSynchronize(cache[i].ready);
        (void)hipEventDestroy(cache[i].ready);
        (void)hipFreeAsync(cache[i].p, nullptr);
        cache.erase(cache.begin() + i);
        any = true;
    }
    if (any) {
        (void)hipStreamSynchronize(nullptr);
        (void)hipMemPoolTrimTo(pool, 0);
    }
    return any;
}

void validate_mesh_host(const lspr_surface* surfaces, int n_surf) {
    LSPR_REQUIRE(surfaces && n_surf >= 1, LSPR_E_INVALID, "need at least one surface");
    for (int s = 0; s < n_surf; ++s) {
        const lspr_surface& f = surfaces[s];
        const std::string tag = "surface " + std::to_string(s) + ": ";
        LSPR_REQUIRE(f.vert && f.tri && f.n_vert >= 3 && f.n_tri >= 4, LSPR_E_INVALID,
                     tag + "empty or null arrays");
        // directed edges (a, b) as 64-bit keys; closed + consistently oriented + edge-manifold
        // means every directed edge occurs once and its reverse occurs once
        std::vector<uint64_t> edges;
        edges.reserve(3 * static_cast<size_t>(f.n_tri));
        double vol = 0.0;
        for (int t = 0; t < f.n_tri; ++t) {
            int v[3];
            for (int k = 0; k < 3; ++k) {
                v[k] = f.tri[3 * t + k];
                LSPR_REQUIRE(v[k] >= 0 && v[k] < f.n_vert, LSPR_E_MESH,
                             tag + "vertex index out of range in triangle " + std::to_string(t));
            }
            LSPR_REQUIRE(v[0] != v[1] && v[1] != v[2] && v[0] != v[2], LSPR_E_MESH,
                         tag + "repeated vertex in triangle " + std::to_string(t));
            const double* a = f.vert + 3 * v[0];
            const double* b = f.vert + 3 * v[1];
            const double* c = f.vert + 3 * v[2];
            const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
            const double w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
            const double n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2],
                                 u[0] * w[1] - u[1] * w[0]};
            const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
            const double sc = std::max(u[0] * u[0] + u[1] * u[1] + u[2] * u[2],
                                       w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
            LSPR_REQUIRE(nn > 1e-14 * sc, LSPR_E_MESH,
                         tag + "degenerate triangle " + std::to_string(t));
            vol += (a[0] * n[0] + a[1] * n[1] + a[2] * n[2]) / 6.0;
            for (int k = 0; k < 3; ++k)
                edges.push_back(static_cast<uint64_t>(v[k]) << 32 |
                                static_cast<uint32_t>(v[(k + 1) % 3]));
        }
        std::sort(edges.begin(), edges.end());
        for (size_t k = 1; k < edges.size(); ++k)
            LSPR_REQUIRE(edges[k] != edges[k - 1], LSPR_E_MESH,
                         tag + "edge used twice in the same direction (orientation or "
                               "non-manifold)");
        for (uint64_t e : edges) {
            const uint64_t r = (e & 0xffffffffull) << 32 | (e >> 32);
            LSPR_REQUIRE(std::binary_search(edges.begin(), edges.end(), r), LSPR_E_MESH,
                         tag + "open surface (edge without its reverse)");
        }
        LSPR_REQUIRE(vol > 0.0, LSPR_E_MESH,
                     tag + "negative enclosed volume (normals point inwards)");
    }
}

void validate_op(const lspr_surface* surfaces, int n_surf, const lspr_op_params* op) {
    int64_t N = 0;
    for (int s = 0; s < n_surf; ++s) {
        LSPR_REQUIRE(surfaces[s].vert && surfaces[s].tri && surfaces[s].n_tri > 0 &&
                 surfaces[s].n_vert > 0,
             LSPR_E_INVALID, "empty surface");
        N += surfaces[s].n_tri;
    }
    LSPR_REQUIRE(N < (1ll << 28), LSPR_E_INVALID, "too many panels");
    std::vector<double> b, w;
    LSPR_REQUIRE(lspr::triangle_rule(op->k_far, b, w) && op->k_far <= 8, LSPR_E_INVALID,
             "k_far must be 1, 3, 4 or 7");
    LSPR_REQUIRE(lspr::triangle_rule(op->k_fine, b, w), LSPR_E_INVALID,
             "k_fine must be one of 1, 3, 4, 7, 19, 25, 37");
    LSPR_REQUIRE(op->n_k >= 1 && op->n_k <= 64, LSPR_E_INVALID, "n_k must be in 1..64");
    LSPR_REQUIRE(op->threshold > 0.0, LSPR_E_INVALID, "threshold must be positive");
    LSPR_REQUIRE(op->method == LSPR_DENSE || op->method == LSPR_TREECODE, LSPR_E_INVALID,
             "unknown method");
    LSPR_REQUIRE(op->precision == LSPR_FP32 || op->precision == LSPR_FP64 ||
                     op->precision == LSPR_FP32_REFINE64 || op->precision == LSPR_FP32_LEAD64,
                 LSPR_E_INVALID, "unknown precision");
    if (op->method == LSPR_TREECODE) {
        LSPR_REQUIRE(op->p == 2 || op->p == 4 || op->p == 6 || op->p == 8 || op->p == 10 ||
                         op->p == 12 || op->p == 15,
                     LSPR_E_INVALID, "p must be 2, 4, 6, 8, 10, 12 or 15");
        LSPR_REQUIRE(op->p <= 10 || (op->flags & LSPR_NO_MATRIX_CORES) == 0, LSPR_E_INVALID,
                     "expansion orders above 10 run only on matrix cores");
        LSPR_REQUIRE(op->theta > 0.0 && op->theta < 1.0, LSPR_E_INVALID,
             "theta must be in (0, 1)");
    }
    LSPR_REQUIRE(op->ncrit >= 0 && op->m2p_min_panels >= 0, LSPR_E_INVALID,
             "ncrit and m2p_min_panels must be >= 0");
    LSPR_REQUIRE((op->flags & ~(LSPR_NO_MATRIX_CORES | LSPR_STREAM_NARROW | LSPR_PAIR_OPERATORS |
                                LSPR_PAIR_NARROW | LSPR_FOUR_WAVE)) == 0,
                 LSPR_E_INVALID, "unknown flags");
}

void validate_gmres(const lspr_gmres_params& gm, int precision) {
    LSPR_REQUIRE(gm.tol > 0.0 && gm.restart >= 1 && gm.restart <= 512 && gm.max_iter >= 1 &&
                     gm.inner_tol >= 0.0 && gm.inner_tol < 1.0 &&
                     (gm.precond == 0 || gm.precond == 1),
                 LSPR_E_INVALID, "bad GMRES parameters");
    if (precision == LSPR_FP32 || precision == LSPR_FP32_LEAD64)
        LSPR_REQUIRE(gm.tol >= FP32_MIN_TOL, LSPR_E_INVALID,
                     "tol below 1e-6 cannot be certified with FP32 products; use "
                     "LSPR_FP32_REFINE64 (FP64 residuals) or LSPR_FP64");
    if (precision == LSPR_FP32_REFINE64)
        LSPR_REQUIRE(gm.inner_tol == 0.0 || gm.inner_tol >= FP32_MIN_TOL, LSPR_E_INVALID,
                     "inner_tol below 1e-6 cannot be reached by the FP32 inner solves");
}

void create_geometry(Geometry& g, const lspr_surface* surfaces, int n_surf,
                     const lspr_op_params& opr, hipStream_t stream) {
    const lspr_op_params* op = &opr;
    validate_op(surfaces, n_surf, op);
    g.stream = static_cast<hipStream_t>(stream);
    g.K = op->k_far;
    g.Kf = op->k_fine;
    g.Nk = op->n_k;
    g.threshold = op->threshold;
    g.method = op->method;
    g.P = op->method == LSPR_TREECODE ? op->p : 4;
    g.theta = op->theta;
    g.ncrit = op->ncrit > 0 ? op->ncrit : 16;
    g.precision = op->precision;
    g.need32 = op->precision != LSPR_FP64;
    g.need64 = op->precision != LSPR_FP32;
    g.n_terms = lspr::expansion_terms(g.P);
    g.m2p_min_panels = op->m2p_min_panels > 0 ? op->m2p_min_panels : g.n_terms;
    g.allow_mfma = (op->flags & LSPR_NO_MATRIX_CORES) == 0;
    g.stream_narrow = (op->flags & LSPR_STREAM_NARROW) != 0;
    g.pair_ops = (op->flags & LSPR_PAIR_OPERATORS) != 0;
    g.pair_narrow = (op->flags & LSPR_PAIR_NARROW) != 0;
    g.four_wave = (op->flags & LSPR_FOUR_WAVE) != 0;
    lspr::prof::Scope setup_scope("setup", g.stream, 0.0, 0.0);
    lspr::build_geometry(g, surfaces, n_surf);
    lspr::build_tree(g);
    lspr::build_lists(g);
    // boxes whose moments are needed, and the row block of each in the moment array
    // (in box order: a flag per box, then the flagged boxes numbered)
    g.mom_slot_h.assign(g.n_boxes, -1);
    for (int32_t b : g.m2p_box_h) g.mom_slot_h[b] = 0;
    g.mom_boxes.clear();
    for (int32_t b = 0; b < g.n_boxes; ++b)
        if (g.mom_slot_h[b] == 0) {
            g.mom_slot_h[b] = static_cast<int32_t>(g.mom_boxes.size());
            g.mom_boxes.push_back(b);
        }
    if (g.tile_budget_bytes <= 0.0) {
        size_t free_b = 0, total_b = 0;
        LSPR_HIP(hipMemGetInfo(&free_b, &total_b));
        // free memory plus what the library's pool holds for reuse (cached blocks and reserved
        // memory not in use: an allocation that does not fit returns them first).  Both stores
        // of the 491k-panel sensor (48 + 96 GB at P = 10) fit on one MI355X beside its Krylov
        // state (15 GB at 16 wavelengths).
        const size_t avail = free_b + lspr::reusable_bytes(lspr::alloc_ctx().pool);
        g.tile_budget_bytes = 0.55 * static_cast<double>(std::min(avail, total_b));
    }
    // no tile plan when not even one store of a needed precision fits (e.g. every pair of a
    // large mesh summed directly): the products then run on the vector ALUs
    bool tiles = g.allow_mfma;
    if (tiles) {
        const double elems = static_cast<double>(lspr::estimate_tile_elems(g));
        tiles = (g.need32 && 4.0 * elems <= g.tile_budget_bytes) ||
                (g.need64 && 8.0 * elems <= g.tile_budget_bytes);
        LSPR_REQUIRE(tiles || g.P <= 10, LSPR_E_NOMEM,
                     "expansion orders above 10 run only from matrix-core tiles, and they do not "
                     "fit the tile budget");
    }
    // the host part of the tiles runs beside the moment set-up and the near-singular table
    std::unique_ptr<lspr::TilePlan> plan_buf;
    std::future<void> plan;
    if (tiles) {
        plan_buf = lspr::take_plan();
        plan = std::async(std::launch::async,
                          [&g, p = plan_buf.get()] { lspr::plan_tiles(g, *p); });
    }
    if (!g.mom_boxes.empty()) {
        const std::vector<lspr::Range>& bh = g.box_rng_h;
        g.mom_panels = 0;
        for (int32_t b : g.mom_boxes) g.mom_panels += bh[b].end - bh[b].start;
        // P2M work items: segments of at most 128 panels per expanded box
        constexpr int SEG = 128;
        std::vector<lspr::P2MSeg> segs;
        std::vector<lspr::P2MRed> reds;
        int slots = 0;
        for (int32_t b : g.mom_boxes) {
            const int n = bh[b].end - bh[b].start;
            const int ns = (n + SEG - 1) / SEG;
            const int slot0 = ns > 1 ? slots : -1;
            const int ms = g.mom_slot_h[b];
            for (int k = 0; k < ns; ++k)
                segs.push_back({b, bh[b].start + k * SEG, std::min(bh[b].end, bh[b].start + (k + 1) * SEG),
                                ns > 1 ? slots + k : -1, ms});
            if (ns > 1) {
                reds.push_back({b, slot0, slot0 + ns, ms});
                slots += ns;
            }
        }
        g.n_seg = static_cast<int>(segs.size());
        g.n_slots = slots;
        g.n_red = static_cast<int>(reds.size());
        g.p2m_seg.alloc(segs.size());
        g.mom_slot.alloc(g.n_boxes);
        lspr::Uploads up(g.stream);
        up.add(g.p2m_seg.p, segs.data(), segs.size());
        up.add(g.mom_slot.p, g.mom_slot_h.data(), g.mom_slot_h.size());
        if (!reds.empty()) {
            g.p2m_red.alloc(reds.size());
            up.add(g.p2m_red.p, reds.data(), reds.size());
        }
        up.flush();
        g.p2m_seg_h = std::move(segs);
    }
    lspr::build_near_table(g);
    if (tiles) {
        plan.get();
        lspr::build_tiles(g, *plan_buf);
        lspr::put_plan(std::move(plan_buf));
    }
    lspr::precompute_rhs(g);
    // the host copies were only needed while building
    g.box_rng_h = {};
    g.p2p_rng_h = {};
    g.m2p_off_h = {};
    g.p2p_off_h = {};
    g.m2p_self_h = {};
    g.p2p_self_h = {};
    g.m2p_box_h = {};
    g.p2m_seg_h = {};
    g.mom_slot_h = {};
}

bool solve_geometry(Geometry& g, int n_lambda, const double* lambda_nm,
                    const lspr_c64* eps_medium, const lspr_c64* eps_surface,
                    const double* e_field, const lspr_gmres_params& gmr, hipStream_t stream,
                    lspr_c64* phi, lspr_c64* dphi, lspr_c64* p_sensor, lspr_c64* p_total,
                    double* cext_sensor, double* cext_total, int32_t* iters, double* rel_resid) {
    const lspr_gmres_params* gm = &gmr;
    LSPR_REQUIRE(lambda_nm && eps_medium && eps_surface && e_field && gm && n_lambda >= 1,
                 LSPR_E_INVALID, "bad arguments");
    validate_gmres(*gm, g.precision);
    const double e2 = e_field[0] * e_field[0] + e_field[1] * e_field[1] + e_field[2] * e_field[2];
    LSPR_REQUIRE(e2 > 0.0, LSPR_E_INVALID, "zero incident field");
    for (int k = 0; k < n_lambda; ++k)
        LSPR_REQUIRE(lambda_nm[k] > 0.0, LSPR_E_INVALID, "wavelengths must be positive");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t nvec = 2 * static_cast<int64_t>(g.N);
    bool all_ok = true;
    for (int b0 = 0; b0 < n_lambda; b0 += MAX_BATCH) {
        const int B = std::min(MAX_BATCH, n_lambda - b0);
        const lspr::EpsSet e = make_eps(B, g.S, eps_medium + b0, eps_surface + b0 * g.S);
        lspr::DevBuf<double2> ratio, xs(B * nvec);
        lspr::upload_ratios(g, e, B, ratio, s);
        const lspr::SolveResult r =
            g.precision == LSPR_FP32_REFINE64
                ? lspr::refine_solve(g, B, ratio.p, e_field, *gm, xs.p, s)
                : lspr::gmres_solve(g, g.precision, B, ratio.p, e_field, *gm, nullptr, xs.p, s);
        all_ok = all_ok && r.all_converged;
        std::vector<double> q;
        lspr::dipole_moments(g, B, ratio.p, e_field, xs.p, q, s);
        for (int b = 0; b < B; ++b) {
            const int k = b0 + b;
            const std::complex<double> em(eps_medium[k].re, eps_medium[k].im);
            const std::complex<double> kw = 2.0 * M_PI * std::sqrt(em) / lambda_nm[k];
            for (int which = 0; which < 2; ++which) {
                std::complex<double> qv[3];
                for (int d = 0; d < 3; ++d)
                    qv[d] = std::complex<double>(q[b * 12 + 6 * which + 2 * d],
                                                 q[b * 12 + 6 * which + 2 * d + 1]);
                const std::complex<double> eq = e_field[0] * qv[0] + e_field[1] * qv[1] +
                                                e_field[2] * qv[2];
                const double cext = std::imag(kw * kw * eq) / (kw.real() * e2);
                lspr_c64* pp = which == 0 ? p_sensor : p_total;
                double* cc = which == 0 ? cext_sensor : cext_total;
                if (pp)
                    for (int d = 0; d < 3; ++d) {
                        const std::complex<double> p = em * qv[d];
                        pp[3 * k + d] = lspr_c64{p.real(), p.imag()};
                    }
                if (cc) cc[k] = cext;
            }
            if (iters) iters[k] = r.iters[b];
            if (rel_resid) rel_resid[k] = r.rel_resid[b];
        }
        if (phi || dphi)
            lspr::unpermute(g, B, xs.p, phi ? reinterpret_cast<double2*>(phi) + b0 * g.N : nullptr,
                            dphi ? reinterpret_cast<double2*>(dphi) + b0 * g.N : nullptr, s);
        LSPR_HIP(hipStreamSynchronize(s));
    }
    return all_ok;
}

int64_t solve_bytes(int64_t N, int S, int B, const lspr_op_params& op,
                    const lspr_gmres_params& gm) {
    const int64_t nvec = 2 * N, m1 = gm.restart + 1;
    const int64_t esz = op.precision == LSPR_FP32 ? 4 : 8;  // largest product precision
    const int64_t pad = (2 * B + 15) / 16 * 16;
    const int64_t nblk = (nvec + 4095) / 4096 + 1;  // Arnoldi blocks of 4096 elements
    int64_t b = 0;
    b += static_cast<int64_t>(B) * m1 * nvec * 16;                 // Krylov basis
    b += static_cast<int64_t>(B) * nvec * 16 * 3;                  // x, w, b
    // partial inner products (one per wave of each block), Hessenberg matrices, coefficients
    b += static_cast<int64_t>(B) * (2 * m1 + 3) * 4 * nblk * 16;
    b += 2 * static_cast<int64_t>(B) * m1 * m1 * 16 + static_cast<int64_t>(B) * (8 * m1 + 64) * 16;
    if (op.precision == LSPR_FP32_REFINE64)
        b += static_cast<int64_t>(B) * nvec * 16 * 4;              // refinement b, r, d, w
    b += N * 2 * pad * esz;                                        // packed densities
    b += N * 2 * pad * 8 * (S > 1 ? 2 : 1);                        // raw layer sums
    // moments and P2M partial sums: expanded boxes hold at most N panels per tree level
    const int64_t terms = static_cast<int64_t>(op.p + 1) * (op.p + 1);
    int levels = 2;
    for (int64_t n = N; n > terms; n /= 4) ++levels;
    const int64_t rows = levels * (N / std::max<int64_t>(terms, 1) + S) * terms;
    b += 2 * rows * 2 * pad * esz;
    return b;
}

int64_t tile_cap_bytes(int64_t N, const lspr_op_params& op) {
    const int precision = op.precision;
    const int64_t per_elem = (precision != LSPR_FP64 ? 4 : 0) + (precision != LSPR_FP32 ? 8 : 0);
    // 24 K elements per panel at P <= 8 (measured: 13-18 K), more with more Taylor terms
    const int64_t terms = static_cast<int64_t>(op.p + 1) * (op.p + 1);
    return N * 24 * 1024 * std::max<int64_t>(terms, 81) / 81 * per_elem;
}

int64_t request_footprint(int64_t N, int S, int n_lambda, const lspr_op_params& op,
                          const lspr_gmres_params& gm) {
    const int B = std::min(n_lambda, MAX_BATCH);
    const int64_t esz = op.precision == LSPR_FP32 ? 4 : 8;
    // mesh upload, sorted panel data, tree, lists and near-singular table (up to 96 pairs per
    // target), the set-up temporaries, and the right-hand-side columns
    int64_t b = N * (1024 + 24 * S + (4 + 4 * op.k_far) * esz + 96 * 20) + (64 << 20);
    b += N * 32 * (esz + 16);
    if ((op.flags & LSPR_NO_MATRIX_CORES) == 0)
        b += tile_cap_bytes(N, op);
    return b + solve_bytes(N, S, B, op, gm);
}

}  // namespace lspr

size_t lspr::Geometry::device_bytes() const {
    return tri.bytes() + cen.bytes() + nrm.bytes() + area.bytes() + surf.bytes() + perm.bytes() +
           iperm.bytes() + morton.bytes() + boxes.bytes() + far_rule.bytes() +
           mom_slot.bytes() + chunks.bytes() + m2p_off.bytes() + m2p_box.bytes() +
           m2p_self.bytes() + p2p_off.bytes() + p2p_rng.bytes() + p2p_self.bytes() +
           near_off64.bytes() + near_col.bytes() + near_dv.bytes() + near_dk.bytes() +
           vself.bytes() + rhs_u.bytes() + charge_u.bytes() + ws_inv_eps.bytes() + ws_dens.bytes() + ws_mom.bytes() + ws_out.bytes() +
           ws_part.bytes() + p2m_seg.bytes() + p2m_red.bytes() + p2mA.bytes() + p2mA64.bytes() + p2m_aoff.bytes() + tiles.bytes() + tile_off.bytes() + chunk_order.bytes() +
           far_plan[0].bytes() + far_plan[1].bytes() + far_plan[2].bytes() + ws_fpart.bytes() +
           tile_self.bytes() + tileA.bytes() + tileA64.bytes() + src32.bytes() + src64.bytes();
}

extern "C" {

const char* lspr_status_string(int code) {
    switch (code) {
        case LSPR_OK: return "ok";
        case LSPR_E_INVALID: return "invalid argument";
        case LSPR_E_MESH: return "invalid mesh";
        case LSPR_E_NOMEM: return "out of memory";
        case LSPR_E_DEVICE: return "device error";
        case LSPR_E_NOCONV: return "GMRES did not converge";
        case LSPR_E_BUSY: return "busy";
        default: return "unknown status";
    }
}

const char* lspr_last_error(void) { return lspr::last_error().c_str(); }

int lspr_triangle_rule(int32_t n, double* bary, double* w) {
    return guarded([&] {
        LSPR_REQUIRE(bary && w, LSPR_E_INVALID, "null output");
        std::vector<double> b, ww;
        LSPR_REQUIRE(lspr::triangle_rule(n, b, ww), LSPR_E_INVALID, "no rule with that many points");
        std::copy(b.begin(), b.end(), bary);
        std::copy(ww.begin(), ww.end(), w);
        return LSPR_OK;
    });
}

int lspr_gauss_legendre(int32_t n, double* t, double* w) {
    return guarded([&] {
        LSPR_REQUIRE(t && w && n >= 1 && n <= 256, LSPR_E_INVALID, "bad Gauss-Legendre request");
        std::vector<double> a, b;
        lspr::gauss_legendre(n, a, b);
        std::copy(a.begin(), a.end(), t);
        std::copy(b.begin(), b.end(), w);
        return LSPR_OK;
    });
}

int lspr_resonance_peak(int32_t n, const double* lambda, const double* cext,
                        double* peak_lambda, double* peak_cext) {
    return guarded([&] {
        LSPR_REQUIRE(n >= 3 && lambda && cext && peak_lambda && peak_cext, LSPR_E_INVALID,
                     "need at least three samples and non-null pointers");
        for (int k = 1; k < n; ++k)
            LSPR_REQUIRE(lambda[k] > lambda[k - 1], LSPR_E_INVALID,
                         "wavelengths must be strictly increasing");
        int m = 0;
        for (int k = 1; k < n; ++k)
            if (cext[k] > cext[m]) m = k;
        if (m == 0 || m == n - 1) {
            *peak_lambda = lambda[m];
            *peak_cext = cext[m];
            return LSPR_OK;
        }
        // parabola c(x) = y1 + a (x - x1) + b (x - x1)^2 through (x0, y0), (x1, y1), (x2, y2)
        const double x0 = lambda[m - 1], x1 = lambda[m], x2 = lambda[m + 1];
        const double y0 = cext[m - 1], y1 = cext[m], y2 = cext[m + 1];
        const double h0 = x0 - x1, h2 = x2 - x1;
        const double s0 = (y0 - y1) / h0, s2 = (y2 - y1) / h2;  // secant slopes
        const double b = (s2 - s0) / (h2 - h0);
        const double a = s0 - b * h0;
        if (!(b < 0.0)) {  // flat or convex around the sample: keep the sample
            *peak_lambda = x1;
            *peak_cext = y1;
            return LSPR_OK;
        }
        const double dx = -a / (2.0 * b);
        *peak_lambda = x1 + dx;
        *peak_cext = y1 + a * dx + b * dx * dx;
        return LSPR_OK;
    });
}

int lspr_mesh_validate(const lspr_surface* surfaces, int32_t n_surf) {
    return guarded([&] {
        lspr::validate_mesh_host(surfaces, n_surf);
        return LSPR_OK;
    });
}

int lspr_geometry_create(const lspr_surface* surfaces, int32_t n_surf, const lspr_op_params* op,
                         void* stream, lspr_geometry** out) {
    return guarded([&] {
        LSPR_REQUIRE(surfaces && op && out && n_surf >= 1 && n_surf <= 4096, LSPR_E_INVALID,
                     "bad arguments");
        *out = nullptr;
        auto h = std::make_unique<lspr_geometry>();
        lspr::PoolScope ps(static_cast<hipStream_t>(stream));
        lspr::create_geometry(h->g, surfaces, n_surf, *op, static_cast<hipStream_t>(stream));
        *out = h.release();
        return LSPR_OK;
    });
}

int lspr_geometry_destroy(lspr_geometry* g) {
    return guarded([&] {
        if (g) {
            (void)hipStreamSynchronize(g->g.stream);
            lspr::PoolScope ps(g->g.stream);  // pooled memory goes back on the geometry's stream
            delete g;
        }
        return LSPR_OK;
    });
}

int lspr_geometry_set_charges(lspr_geometry* h, int32_t n_q, const double* pos, const double* q,
                              const int32_t* surface, void* stream) {
    return guarded([&] {
        LSPR_REQUIRE(h && n_q >= 0 && (n_q == 0 || (pos && q && surface)), LSPR_E_INVALID,
                     "bad arguments");
        hipStream_t s = static_cast<hipStream_t>(stream);
        lspr::PoolScope ps(s);
        lspr::set_charges(h->g, n_q, pos, q, surface, s);
        return LSPR_OK;
    });
}

int lspr_geometry_info(const lspr_geometry* h, lspr_geometry_stats* o) {
    return guarded([&] {
        LSPR_REQUIRE(h && o, LSPR_E_INVALID, "null argument");
        const lspr::Geometry& g = h->g;
        o->n_panels = g.N;
        o->n_surfaces = g.S;
        o->n_nodes = static_cast<int64_t>(g.N) * g.K;
        o->n_boxes = g.n_boxes;
        o->n_leaves = g.n_leaves;
        o->n_target_chunks = g.n_chunks;
        o->n_m2p = g.n_m2p;
        o->n_p2p_ranges = g.n_p2p;
        o->p2p_pairs = g.p2p_pairs;
        o->m2p_pairs = g.m2p_pairs;
        o->n_near = g.n_near;
        o->device_bytes = static_cast<int64_t>(g.device_bytes());
        o->n_terms = g.n_terms;
        o->ncrit = g.ncrit;
        o->target_chunk = g.tchunk;
        o->max_depth = g.max_depth;
        o->n_tiles = g.n_tiles;
        o->tile_steps = g.tile_steps;
        o->max_chunk_steps = g.max_chunk_steps;
        return LSPR_OK;
    });
}

int lspr_apply(lspr_geometry* h, int32_t n_cols, const lspr_c64* eps_medium,
               const lspr_c64* eps_surface, const lspr_c64* x, lspr_c64* y, void* stream) {
    return guarded([&] {
        LSPR_REQUIRE(h && eps_medium && eps_surface && x && y && n_cols >= 1, LSPR_E_INVALID,
                     "bad arguments");
        lspr::Geometry& g = h->g;
        hipStream_t s = static_cast<hipStream_t>(stream);
        lspr::PoolScope ps(s);
        const int64_t nvec = 2 * static_cast<int64_t>(g.N);
        for (int b0 = 0; b0 < n_cols; b0 += MAX_BATCH) {
            const int B = std::min(MAX_BATCH, n_cols - b0);
            const lspr::EpsSet e = make_eps(B, g.S, eps_medium + b0, eps_surface + b0 * g.S);
            lspr::DevBuf<double2> ratio, xs(B * nvec), ys(B * nvec);
            lspr::upload_ratios(g, e, B, ratio, s);
            lspr::to_sorted(g, B, reinterpret_cast<const double2*>(x) + b0 * nvec, xs.p, s);
            lspr::system_apply(g, g.need64 ? LSPR_FP64 : LSPR_FP32, B, ratio.p, xs.p, nvec, ys.p,
                               nvec, nullptr, s);
            lspr::from_sorted(g, B, ys.p, reinterpret_cast<double2*>(y) + b0 * nvec, s);
            LSPR_HIP(hipStreamSynchronize(s));
        }
        return LSPR_OK;
    });
}

int lspr_rhs(lspr_geometry* h, int32_t n_cols, const lspr_c64* eps_medium,
             const lspr_c64* eps_surface, const double* e_field, lspr_c64* b, void* stream) {
    return guarded([&] {
        LSPR_REQUIRE(h && eps_medium && eps_surface && e_field && b && n_cols >= 1,
                     LSPR_E_INVALID, "bad arguments");
        lspr::Geometry& g = h->g;
        hipStream_t s = static_cast<hipStream_t>(stream);
        lspr::PoolScope ps(s);
        const int64_t nvec = 2 * static_cast<int64_t>(g.N);
        for (int b0 = 0; b0 < n_cols; b0 += MAX_BATCH) {
            const int B = std::min(MAX_BATCH, n_cols - b0);
            const lspr::EpsSet e = make_eps(B, g.S, eps_medium + b0, eps_surface + b0 * g.S);
            lspr::DevBuf<double2> ratio, bs(B * nvec);
            lspr::upload_ratios(g, e, B, ratio, s);
            lspr::system_rhs(g, B, ratio.p, e_field, bs.p, nvec, s);
            lspr::from_sorted(g, B, bs.p, reinterpret_cast<double2*>(b) + b0 * nvec, s);
            LSPR_HIP(hipStreamSynchronize(s));
        }
        return LSPR_OK;
    });
}

int lspr_autotune(const lspr_surface* surfaces, int32_t n_surf, int32_t n_cols,
                  const lspr_c64* eps_medium, const lspr_c64* eps_surface, double max_rel_err,
                  lspr_op_params* op, lspr_tune_entry* entries, int32_t max_entries,
                  int32_t* n_entries, void* stream) {
    return guarded([&] {
        LSPR_REQUIRE(surfaces && op && eps_medium && eps_surface && n_entries && n_surf >= 1 &&
                         n_cols >= 1 && n_cols <= MAX_BATCH && max_rel_err > 0.0 &&
                         max_entries >= 0 && (entries != nullptr || max_entries == 0),
                     LSPR_E_INVALID, "bad arguments");
        hipStream_t s = static_cast<hipStream_t>(stream);
        lspr::PoolScope ps(s);
        int64_t N = 0;
        for (int k = 0; k < n_surf; ++k) N += surfaces[k].n_tri;
        const int64_t nvec = 2 * N;
        // probe vector in caller order: a fixed linear congruential sequence in [-1, 1)
        std::vector<double2> xh(nvec);
        uint64_t st = 0x9e3779b97f4a7c15ull;
        auto uni = [&] {
            st = st * 6364136223846793005ull + 1442695040888963407ull;
            return static_cast<double>(st >> 11) * (2.0 / 9007199254740992.0) - 1.0;
        };
        for (auto& v : xh) {
            v.x = uni();
            v.y = uni();
        }
        lspr::DevBuf<double2> x(nvec), y(nvec), yref(nvec);
        LSPR_HIP(hipMemcpyAsync(x.p, xh.data(), nvec * sizeof(double2), hipMemcpyHostToDevice, s));
        std::vector<lspr_c64> em(n_cols, eps_medium[0]), es;
        for (int c = 0; c < n_cols; ++c)
            for (int k = 0; k < n_surf; ++k) es.push_back(eps_surface[k]);
        const lspr::EpsSet e1 = make_eps(1, n_surf, em.data(), es.data());
        const lspr::EpsSet eb = make_eps(n_cols, n_surf, em.data(), es.data());
        // product of the probe vector in precision prec (caller order)
        auto product = [&](lspr::Geometry& g, int prec, double2* out) {
            lspr::DevBuf<double2> ratio, xs(nvec), ys(nvec);
            lspr::upload_ratios(g, e1, 1, ratio, s);
            lspr::to_sorted(g, 1, x.p, xs.p, s);
            lspr::system_apply(g, prec, 1, ratio.p, xs.p, nvec, ys.p, nvec, nullptr, s);
            lspr::from_sorted(g, 1, ys.p, out, s);
            LSPR_HIP(hipStreamSynchronize(s));
        };
        std::vector<double2> yh(nvec), rh(nvec);
        {
            // reference: every far pair summed directly in FP64 (on matrix cores when its tiles
            // fit, otherwise by the vector-ALU kernel)
            lspr_op_params r = *op;
            r.precision = LSPR_FP64;
            r.method = LSPR_DENSE;
            lspr::Geometry gr;
            lspr::create_geometry(gr, surfaces, n_surf, r, s);
            product(gr, LSPR_FP64, yref.p);
        }
        LSPR_HIP(hipMemcpy(rh.data(), yref.p, nvec * sizeof(double2), hipMemcpyDeviceToHost));
        double rn = 0.0;
        for (const auto& v : rh) rn += v.x * v.x + v.y * v.y;
        rn = std::sqrt(rn);
        LSPR_REQUIRE(rn > 0.0, LSPR_E_INVALID, "zero reference product");
        const int tprec = op->precision == LSPR_FP64 ? LSPR_FP64 : LSPR_FP32;
        hipEvent_t e0 = nullptr, e_1 = nullptr;
        LSPR_HIP(hipEventCreate(&e0));
        LSPR_HIP(hipEventCreate(&e_1));
        struct Events {
            hipEvent_t a, b;
            ~Events() {
                (void)hipEventDestroy(a);
                (void)hipEventDestroy(b);
            }
        } events{e0, e_1};
        int count = 0;
        auto record = [&](const lspr_tune_entry& t) {
            if (count < max_entries) entries[count] = t;
            ++count;
        };
        // FP64 error of a candidate against the reference, and (if within the bound) its
        // fastest product of n_cols columns in the timed precision, of three after a warm-up
        auto measure = [&](const lspr_op_params& c, bool timed) {
            lspr_tune_entry t{c.p, c.ncrit, c.theta, 0.0, -1.0, c.m2p_min_panels, c.flags};
            lspr_op_params cc = c;
            cc.method = LSPR_TREECODE;
            // both tile stores: FP64 for the error, the timed precision for speed
            cc.precision = tprec == LSPR_FP64 ? LSPR_FP64 : LSPR_FP32_LEAD64;
            lspr::Geometry g;
            try {
                lspr::create_geometry(g, surfaces, n_surf, cc, s);
            } catch (const lspr::Error& err) {
                // a candidate whose set-up does not fit the device is skipped (rel_err infinite)
                if (err.code != LSPR_E_NOMEM) throw;
                (void)hipGetLastError();
                LSPR_HIP(hipStreamSynchronize(s));
                t.rel_err = HUGE_VAL;
                return t;
            }
            product(g, LSPR_FP64, y.p);
            LSPR_HIP(hipMemcpy(yh.data(), y.p, nvec * sizeof(double2), hipMemcpyDeviceToHost));
            double dn = 0.0;
            for (int64_t i = 0; i < nvec; ++i) {
                const double dx = yh[i].x - rh[i].x, dy = yh[i].y - rh[i].y;
                dn += dx * dx + dy * dy;
            }
            t.rel_err = std::sqrt(dn) / rn;
            if (timed && t.rel_err <= max_rel_err) {
                lspr::DevBuf<double2> ratio, ys(n_cols * nvec), xs(nvec);
                lspr::upload_ratios(g, eb, n_cols, ratio, s);
                lspr::to_sorted(g, 1, x.p, xs.p, s);
                float ms_min = 1e30f;
                for (int rep = 0; rep < 4; ++rep) {
                    LSPR_HIP(hipEventRecord(e0, s));
                    // every column multiplies the same vector (stride 0)
                    lspr::system_apply(g, tprec, n_cols, ratio.p, xs.p, 0, ys.p, nvec, nullptr,
                                       s);
                    LSPR_HIP(hipEventRecord(e_1, s));
                    LSPR_HIP(hipEventSynchronize(e_1));
                    float ms = 0.0f;
                    LSPR_HIP(hipEventElapsedTime(&ms, e0, e_1));
                    if (rep > 0) ms_min = std::min(ms_min, ms);
                }
                t.ms_per_product = ms_min;
            }
            LSPR_HIP(hipStreamSynchronize(s));
            return t;
        };
        // stage 1: expansion order, acceptance parameter and leaf size (large meshes search a
        // narrower grid: each candidate is a full set-up)
        const bool big = N > 100000;
        const std::vector<double> thetas = big ? std::vector<double>{0.5, 0.6}
                                               : std::vector<double>{0.4, 0.5, 0.6, 0.7};
        const std::vector<int> leaves = big ? std::vector<int>{16} : std::vector<int>{8, 16, 32};
        const int orders[] = {4, 6, 8, 10, 12, 15};
        lspr_tune_entry best{0, 0, 0.0, 0.0, -1.0, 0, 0}, closest{0, 0, 0.0, 1e300, -1.0, 0, 0};
        for (double th : thetas)
            for (int nc : leaves)
                for (int P : orders) {
                    lspr_op_params c = *op;
                    c.p = P;
                    c.theta = th;
                    c.ncrit = nc;
                    c.m2p_min_panels = 0;
                    const lspr_tune_entry t = measure(c, true);
                    if (t.ms_per_product >= 0.0 &&
                        (best.ms_per_product < 0.0 || t.ms_per_product < best.ms_per_product))
                        best = t;
                    if (t.rel_err < closest.rel_err) closest = t;
                    record(t);
                    // a higher order only costs more (and one that did not fit, more memory)
                    if (t.rel_err <= max_rel_err || t.rel_err == HUGE_VAL) break;
                }
        // stage 2: the kernel schedule of the best expansion: the cost threshold for expanding a
        // box (half and twice the default of one panel per Taylor term; it moves work between
        // expansions and direct sums, so the bound is checked again), both operators staged once
        // in eight-wave workgroups, for narrow products operands streamed or staged, and for
        // FP32 products the four-wave workgroups that stage the left factors through registers
        if (best.ms_per_product >= 0.0) {
            const int terms = (best.p + 1) * (best.p + 1);
            lspr_op_params b = *op;
            b.p = best.p;
            b.theta = best.theta;
            b.ncrit = best.ncrit;
            b.m2p_min_panels = 0;
            b.flags = op->flags & LSPR_NO_MATRIX_CORES;
            std::vector<lspr_op_params> sched;
            for (int mp : {terms / 2, 2 * terms}) {
                lspr_op_params c = b;
                c.m2p_min_panels = mp;
                sched.push_back(c);
            }
            if (n_cols > 16) {
                lspr_op_params c = b;
                c.flags |= LSPR_PAIR_OPERATORS;
                sched.push_back(c);
            }
            if (n_cols <= 16) {
                lspr_op_params c = b;
                c.flags |= LSPR_STREAM_NARROW;
                sched.push_back(c);
            }
            if (b.precision != LSPR_FP64) {
                lspr_op_params c = b;
                c.flags |= LSPR_FOUR_WAVE;
                sched.push_back(c);
            }
            for (const lspr_op_params& c : sched) {
                const lspr_tune_entry t = measure(c, true);
                record(t);
                if (t.ms_per_product >= 0.0 && t.ms_per_product < best.ms_per_product) best = t;
            }
        }
        *n_entries = count;
        const lspr_tune_entry& pick = best.ms_per_product >= 0.0 ? best : closest;
        op->method = LSPR_TREECODE;
        op->p = pick.p;
        op->theta = pick.theta;
        op->ncrit = pick.ncrit;
        op->m2p_min_panels = pick.m2p_min_panels;
        op->flags = pick.flags;
        if (best.ms_per_product < 0.0) {
            lspr::last_error() = "no candidate meets the error bound";
            return static_cast<int>(LSPR_E_NOCONV);
        }
        return static_cast<int>(LSPR_OK);
    });
}

int lspr_solve(lspr_geometry* h, int32_t n_lambda, const double* lambda_nm,
               const lspr_c64* eps_medium, const lspr_c64* eps_surface, const double* e_field,
               const lspr_gmres_params* gm, void* stream, lspr_c64* phi, lspr_c64* dphi,
               lspr_c64* p_sensor, lspr_c64* p_total, double* cext_sensor, double* cext_total,
               int32_t* iters, double* rel_resid) {
    return guarded([&] {
        LSPR_REQUIRE(h && gm, LSPR_E_INVALID, "bad arguments");
        lspr::PoolScope ps(static_cast<hipStream_t>(stream));
        const bool ok = lspr::solve_geometry(h->g, n_lambda, lambda_nm, eps_medium, eps_surface,
                                             e_field, *gm, static_cast<hipStream_t>(stream), phi,
                                             dphi, p_sensor, p_total, cext_sensor, cext_total,
                                             iters, rel_resid);
        if (!ok) {
            lspr::last_error() = "some wavelengths reached max_iter before tol";
            return static_cast<int>(LSPR_E_NOCONV);
        }
        return static_cast<int>(LSPR_OK);
    });
}

}  // extern "C"
