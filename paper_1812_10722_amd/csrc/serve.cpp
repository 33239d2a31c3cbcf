// Request server: continuous batching of independent solve requests on one device.
//
// Worker threads (one per slot) each own a non-blocking stream.  A request waits in a FIFO
// queue until a worker is free and its footprint estimate fits beside the reservations of the
// requests already admitted; the worker then uploads the mesh, builds the geometry, solves and
// computes the dipoles and extinction cross-sections, all on its stream, with every device
// allocation taken stream-ordered from the server's memory pool.  Requests on different workers
// run concurrently on the device.  After set-up the reservation shrinks to what the request
// actually holds, so that queued requests are admitted early.
#include <algorithm>
#include <cmath>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "driver.hpp"
#include "system.hpp"

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t id = 0;
    // inputs (host copies)
    std::vector<std::vector<double>> vert;
    std::vector<std::vector<int32_t>> tri;
    lspr_op_params op{};
    lspr_gmres_params gm{};
    std::vector<double> lambda;
    std::vector<lspr_c64> em, es;
    double e[3] = {0, 0, 0};
    std::vector<double> qpos, qval;  // point charges (may be empty): [n][3], [n]
    std::vector<int32_t> qsurf;      // [n] enclosing surface
    int64_t n_panels = 0;
    int S = 0, B = 0;
    int64_t est = 0, reserved = 0;
    // results
    int status = LSPR_OK;
    std::string error;
    std::vector<double> cext_s, cext_t, resid;
    std::vector<lspr_c64> p_s, p_t;
    std::vector<int32_t> iters;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int64_t peak = 0;
    bool done = false;
};

}  // namespace

struct lspr_server {
    int device = 0;
    int64_t budget = 0, reserved = 0, peak_reserved = 0;
    int max_slots = 1;
    hipMemPool_t pool = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::unordered_map<uint64_t, std::shared_ptr<Request>> reqs;
    uint64_t next_id = 1;
    int64_t submitted = 0, completed = 0, active = 0, max_active = 0, violations = 0;
    bool stop = false;
    Clock::time_point t0 = Clock::now();

    double now() const {
        return std::chrono::duration<double>(Clock::now() - t0).count();
    }
    void worker(int w);
    void run(Request& r, hipStream_t s);
};

using lspr::guarded;

void lspr_server::run(Request& r, hipStream_t s) {
    lspr::AllocCtx& ctx = lspr::alloc_ctx();
    const int64_t base = ctx.live;
    ctx.peak = ctx.live;
    try {
        std::vector<lspr_surface> host(r.S), dev(r.S);
        for (int k = 0; k < r.S; ++k)
            host[k] = lspr_surface{static_cast<int32_t>(r.vert[k].size() / 3), r.vert[k].data(),
                                   static_cast<int32_t>(r.tri[k].size() / 3), r.tri[k].data()};
        lspr::validate_mesh_host(host.data(), r.S);
        lspr::Geometry g;
        g.tile_budget_bytes =
            static_cast<double>(lspr::tile_cap_bytes(r.n_panels, r.op));
        {
            std::vector<lspr::DevBuf<double>> vd(r.S);
            std::vector<lspr::DevBuf<int32_t>> td(r.S);
            for (int k = 0; k < r.S; ++k) {
                vd[k].alloc(r.vert[k].size());
                td[k].alloc(r.tri[k].size());
                LSPR_HIP(hipMemcpyAsync(vd[k].p, r.vert[k].data(), vd[k].bytes(),
                                        hipMemcpyHostToDevice, s));
                LSPR_HIP(hipMemcpyAsync(td[k].p, r.tri[k].data(), td[k].bytes(),
                                        hipMemcpyHostToDevice, s));
                dev[k] = lspr_surface{host[k].n_vert, vd[k].p, host[k].n_tri, td[k].p};
            }
            lspr::create_geometry(g, dev.data(), r.S, r.op, s);
        }
        if (!r.qval.empty())
            lspr::set_charges(g, static_cast<int>(r.qval.size()), r.qpos.data(), r.qval.data(),
                              r.qsurf.data(), s);
        // the set-up is done: keep only what the solve still needs reserved
        {
            const int64_t need =
                static_cast<int64_t>(g.device_bytes()) +
                lspr::solve_bytes(r.n_panels, r.S, r.B, r.op, r.gm);
            std::lock_guard<std::mutex> lk(mu);
            if (need < r.reserved) {
                reserved -= r.reserved - need;
                r.reserved = need;
                cv_work.notify_all();
            }
        }
        const int L = static_cast<int>(r.lambda.size());
        r.cext_s.assign(L, 0.0);
        r.cext_t.assign(L, 0.0);
        r.resid.assign(L, 0.0);
        r.iters.assign(L, 0);
        r.p_s.assign(3 * L, lspr_c64{0, 0});
        r.p_t.assign(3 * L, lspr_c64{0, 0});
        const bool ok = lspr::solve_geometry(g, L, r.lambda.data(), r.em.data(), r.es.data(), r.e,
                                             r.gm, s, nullptr, nullptr, r.p_s.data(),
                                             r.p_t.data(), r.cext_s.data(), r.cext_t.data(),
                                             r.iters.data(), r.resid.data());
        r.status = ok ? LSPR_OK : LSPR_E_NOCONV;
        if (!ok) r.error = "some wavelengths reached max_iter before tol";
    } catch (const lspr::Error& e) {
        r.status = e.code;
        r.error = e.what();
    } catch (const std::bad_alloc&) {
        r.status = LSPR_E_NOMEM;
        r.error = "host allocation failed";
    } catch (const std::exception& e) {
        r.status = LSPR_E_INVALID;
        r.error = e.what();
    }
    // every buffer of the request has been released stream-ordered; wait for its work to end
    if (hipStreamSynchronize(s) != hipSuccess && r.status == LSPR_OK) {
        r.status = LSPR_E_DEVICE;
        r.error = "stream synchronisation failed";
    }
    r.peak = ctx.peak - base;
}

void lspr_server::worker(int w) {
    (void)hipSetDevice(device);
    lspr::AllocCtx& ctx = lspr::alloc_ctx();
    ctx.pool = pool;
    ctx.stream = streams[w];
    for (;;) {
        std::shared_ptr<Request> r;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_work.wait(lk, [&] {
                return stop ||
                       (!queue.empty() && (active == 0 || reserved + queue.front()->est <= budget));
            });
            if (stop) return;
            r = queue.front();
            queue.pop_front();
            r->reserved = r->est;
            reserved += r->est;
            peak_reserved = std::max(peak_reserved, reserved);
            ++active;
            max_active = std::max(max_active, active);
            r->t_admit = now();
        }
        // Freed memory stays in the pool for the next request; when the device itself no longer
        // has room for this request's estimate, the pool returns what it holds unused (blocks of
        // earlier requests that another request's sizes cannot reuse would otherwise crowd the
        // device out).
        {
            size_t free_b = 0, total_b = 0;
            if (hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
                static_cast<double>(free_b) < 1.1 * static_cast<double>(r->est))
                (void)hipMemPoolTrimTo(pool, 0);
        }
        run(*r, streams[w]);
        {
            std::lock_guard<std::mutex> lk(mu);
            reserved -= r->reserved;
            r->reserved = 0;
            --active;
            ++completed;
            if (r->peak > r->est) ++violations;
            r->t_done = now();
            r->done = true;
        }
        cv_work.notify_all();
        cv_done.notify_all();
    }
}

extern "C" {

int lspr_request_footprint(int64_t n_panels, int32_t n_surf, int32_t n_lambda,
                           const lspr_op_params* op, const lspr_gmres_params* gm,
                           int64_t* bytes) {
    return guarded([&] {
        LSPR_REQUIRE(op && gm && bytes && n_panels > 0 && n_surf >= 1 && n_lambda >= 1,
                     LSPR_E_INVALID, "bad arguments");
        LSPR_REQUIRE(op->precision >= LSPR_FP64 && op->precision <= LSPR_FP32_LEAD64,
                     LSPR_E_INVALID, "unknown precision");
        *bytes = lspr::request_footprint(n_panels, n_surf, n_lambda, *op, *gm);
        return LSPR_OK;
    });
}

int lspr_server_create(const lspr_server_params* params, lspr_server** out) {
    return guarded([&] {
        LSPR_REQUIRE(params && out, LSPR_E_INVALID, "null argument");
        LSPR_REQUIRE(params->max_slots >= 1 && params->max_slots <= 16 &&
                         params->hbm_budget_bytes >= 0,
                     LSPR_E_INVALID, "max_slots must be in 1..16 and the budget >= 0");
        *out = nullptr;
        auto sv = std::make_unique<lspr_server>();
        LSPR_HIP(hipGetDevice(&sv->device));
        size_t free_b = 0, total_b = 0;
        LSPR_HIP(hipMemGetInfo(&free_b, &total_b));
        sv->budget = params->hbm_budget_bytes > 0
                         ? params->hbm_budget_bytes
                         : static_cast<int64_t>(0.85 * static_cast<double>(free_b));
        sv->max_slots = params->max_slots;
        hipMemPoolProps props{};
        props.allocType = hipMemAllocationTypePinned;
        props.handleTypes = hipMemHandleTypeNone;
        props.location.type = hipMemLocationTypeDevice;
        props.location.id = sv->device;
        LSPR_HIP(hipMemPoolCreate(&sv->pool, &props));
        uint64_t keep = UINT64_MAX;  // keep freed memory in the pool for the next request
        LSPR_HIP(hipMemPoolSetAttribute(sv->pool, hipMemPoolAttrReleaseThreshold, &keep));
        for (int w = 0; w < sv->max_slots; ++w) {
            hipStream_t s = nullptr;
            LSPR_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            sv->streams.push_back(s);
        }
        lspr_server* p = sv.get();
        for (int w = 0; w < p->max_slots; ++w) p->workers.emplace_back([p, w] { p->worker(w); });
        *out = sv.release();
        return LSPR_OK;
    });
}

int lspr_server_submit(lspr_server* sv, const lspr_surface* surfaces, int32_t n_surf,
                       const lspr_op_params* op, int32_t n_lambda, const double* lambda_nm,
                       const lspr_c64* eps_medium, const lspr_c64* eps_surface,
                       const double* e_field, const lspr_gmres_params* gm, uint64_t* ticket) {
    return lspr_server_submit_charges(sv, surfaces, n_surf, op, n_lambda, lambda_nm, eps_medium,
                                      eps_surface, e_field, gm, 0, nullptr, nullptr, nullptr,
                                      ticket);
}

int lspr_server_submit_charges(lspr_server* sv, const lspr_surface* surfaces, int32_t n_surf,
                               const lspr_op_params* op, int32_t n_lambda,
                               const double* lambda_nm, const lspr_c64* eps_medium,
                               const lspr_c64* eps_surface, const double* e_field,
                               const lspr_gmres_params* gm, int32_t n_q, const double* pos,
                               const double* q, const int32_t* surface, uint64_t* ticket) {
    return guarded([&] {
        LSPR_REQUIRE(sv && surfaces && op && lambda_nm && eps_medium && eps_surface && e_field &&
                         gm && ticket && n_surf >= 1 && n_surf <= 4096 && n_lambda >= 1 &&
                         n_q >= 0 && (n_q == 0 || (pos && q && surface)),
                     LSPR_E_INVALID, "bad arguments");
        for (int k = 0; k < n_q; ++k)  // checked here so that a bad charge fails the submit
            LSPR_REQUIRE(surface[k] >= 0 && surface[k] < n_surf && std::isfinite(q[k]) &&
                             std::isfinite(pos[3 * k]) && std::isfinite(pos[3 * k + 1]) &&
                             std::isfinite(pos[3 * k + 2]),
                         LSPR_E_INVALID, "charges must be finite and inside a listed surface");
        lspr::validate_op(surfaces, n_surf, op);
        lspr::validate_gmres(*gm, op->precision);
        auto r = std::make_shared<Request>();
        r->S = n_surf;
        for (int k = 0; k < n_surf; ++k) {
            const lspr_surface& f = surfaces[k];
            r->vert.emplace_back(f.vert, f.vert + 3 * static_cast<size_t>(f.n_vert));
            r->tri.emplace_back(f.tri, f.tri + 3 * static_cast<size_t>(f.n_tri));
            r->n_panels += f.n_tri;
        }
        r->op = *op;
        r->gm = *gm;
        r->lambda.assign(lambda_nm, lambda_nm + n_lambda);
        r->em.assign(eps_medium, eps_medium + n_lambda);
        r->es.assign(eps_surface, eps_surface + static_cast<size_t>(n_lambda) * n_surf);
        for (int d = 0; d < 3; ++d) r->e[d] = e_field[d];
        r->qpos.assign(pos, pos + 3 * static_cast<size_t>(n_q));
        r->qval.assign(q, q + n_q);
        r->qsurf.assign(surface, surface + n_q);
        r->B = std::min<int>(n_lambda, lspr::MAX_BATCH);
        r->est = lspr::request_footprint(r->n_panels, n_surf, n_lambda, *op, *gm);
        if (n_q > 0)  // per-panel charge potential, 1 / eps_s per batch column, charge copies
            r->est += 8 * r->n_panels + 16 * static_cast<int64_t>(r->B) * n_surf + 32ll * n_q +
                      8 * (n_surf + 1);
        std::lock_guard<std::mutex> lk(sv->mu);
        LSPR_REQUIRE(!sv->stop, LSPR_E_INVALID, "server is shutting down");
        LSPR_REQUIRE(r->est <= sv->budget, LSPR_E_NOMEM,
                     "request footprint exceeds the server's device-memory budget");
        r->id = sv->next_id++;
        r->t_submit = sv->now();
        sv->reqs[r->id] = r;
        sv->queue.push_back(r);
        ++sv->submitted;
        *ticket = r->id;
        sv->cv_work.notify_all();
        return LSPR_OK;
    });
}

int lspr_server_poll(lspr_server* sv, uint64_t ticket, int32_t wait, lspr_request_info* info,
                     double* cext_sensor, double* cext_total, lspr_c64* p_sensor,
                     lspr_c64* p_total, int32_t* iters, double* rel_resid) {
    return guarded([&] {
        LSPR_REQUIRE(sv, LSPR_E_INVALID, "null server");
        std::unique_lock<std::mutex> lk(sv->mu);
        auto it = sv->reqs.find(ticket);
        LSPR_REQUIRE(it != sv->reqs.end(), LSPR_E_INVALID, "unknown ticket");
        std::shared_ptr<Request> r = it->second;
        if (!r->done) {
            if (!wait) return static_cast<int>(LSPR_E_BUSY);
            sv->cv_done.wait(lk, [&] { return r->done; });
        }
        const size_t L = r->lambda.size();
        if (r->cext_s.size() == L) {
            if (cext_sensor) std::copy(r->cext_s.begin(), r->cext_s.end(), cext_sensor);
            if (cext_total) std::copy(r->cext_t.begin(), r->cext_t.end(), cext_total);
            if (p_sensor) std::copy(r->p_s.begin(), r->p_s.end(), p_sensor);
            if (p_total) std::copy(r->p_t.begin(), r->p_t.end(), p_total);
            if (iters) std::copy(r->iters.begin(), r->iters.end(), iters);
            if (rel_resid) std::copy(r->resid.begin(), r->resid.end(), rel_resid);
        }
        if (info) {
            info->status = r->status;
            info->n_lambda = static_cast<int32_t>(L);
            info->n_panels = r->n_panels;
            info->t_submit = r->t_submit;
            info->t_admit = r->t_admit;
            info->t_done = r->t_done;
            info->est_bytes = r->est;
            info->peak_bytes = r->peak;
            const size_t ne = std::min(r->error.size(), sizeof(info->error) - 1);
            std::copy(r->error.begin(), r->error.begin() + ne, info->error);
            info->error[ne] = '\0';
        }
        sv->reqs.erase(it);
        return static_cast<int>(LSPR_OK);
    });
}

int lspr_server_stats_get(lspr_server* sv, lspr_server_stats* o) {
    return guarded([&] {
        LSPR_REQUIRE(sv && o, LSPR_E_INVALID, "null argument");
        std::lock_guard<std::mutex> lk(sv->mu);
        o->submitted = sv->submitted;
        o->completed = sv->completed;
        o->queued = static_cast<int64_t>(sv->queue.size());
        o->active = sv->active;
        o->max_active = sv->max_active;
        o->budget_bytes = sv->budget;
        o->reserved_bytes = sv->reserved;
        o->peak_reserved_bytes = sv->peak_reserved;
        o->estimate_violations = sv->violations;
        return LSPR_OK;
    });
}

int lspr_server_destroy(lspr_server* sv) {
    return guarded([&] {
        if (!sv) return LSPR_OK;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            for (auto& r : sv->queue) {
                r->status = LSPR_E_INVALID;
                r->error = "cancelled: server destroyed";
                r->done = true;
            }
            sv->queue.clear();
            // running requests finish first
            sv->cv_done.wait(lk, [&] { return sv->active == 0; });
            sv->stop = true;
        }
        sv->cv_work.notify_all();
        sv->cv_done.notify_all();
        for (auto& t : sv->workers) t.join();
        for (hipStream_t s : sv->streams) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
        if (sv->pool) (void)hipMemPoolDestroy(sv->pool);
        delete sv;
        return LSPR_OK;
    });
}

}  // extern "C"
