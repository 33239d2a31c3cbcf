// Set-up and solve drivers shared by the C entry points (capi.cpp) and the request server
// (serve.cpp).
#pragma once

#include "internal.hpp"

// The opaque handle of the C ABI.
struct lspr_geometry {
    lspr::Geometry g;
};

namespace lspr {

// Detail text of the calling thread's last error (lspr_last_error).
std::string& last_error();

// Runs an entry point body, translating exceptions into status codes and error text.
template <class F>
int guarded(F&& f) {
    try {
        last_error().clear();
        return f();
    } catch (const Error& e) {
        last_error() = e.what();
        return e.code;
    } catch (const std::bad_alloc&) {
        last_error() = "host allocation failed";
        return LSPR_E_NOMEM;
    } catch (const std::exception& e) {
        last_error() = e.what();
        return LSPR_E_INVALID;
    }
}

constexpr int MAX_BATCH = 64;  // wavelengths per block matrix-vector product

// Checks the operator parameters and the surface array shapes (throws Error).
void validate_op(const lspr_surface* surfaces, int n_surf, const lspr_op_params* op);
// Smallest relative residual a solve whose final residual is formed with FP32 products can
// certify (the FP32 rounding of one product is about 1e-7 of its norm, and GMRES stalls a few
// times above it near resonance): tol of LSPR_FP32 and LSPR_FP32_LEAD64, inner_tol of
// LSPR_FP32_REFINE64.
constexpr double FP32_MIN_TOL = 1e-6;
// Checks GMRES parameters against the product precision of the solve (throws Error).
void validate_gmres(const lspr_gmres_params& gm, int precision);
// Host check of closed, consistently oriented, edge-manifold surfaces (throws Error, E_MESH).
void validate_mesh_host(const lspr_surface* surfaces, int n_surf);

// Builds the geometry-only data of a mesh (device vertex and triangle arrays) on stream s.
void create_geometry(Geometry& g, const lspr_surface* dev_surfaces, int n_surf,
                     const lspr_op_params& op, hipStream_t s);

// Solves for n_lambda wavelengths in batches of MAX_BATCH; returns false when some
// wavelength reached max_iter first (outputs are still filled from the last iterate).
bool solve_geometry(Geometry& g, int n_lambda, const double* lambda_nm,
                    const lspr_c64* eps_medium, const lspr_c64* eps_surface,
                    const double* e_field, const lspr_gmres_params& gm, hipStream_t s,
                    lspr_c64* phi, lspr_c64* dphi, lspr_c64* p_sensor, lspr_c64* p_total,
                    double* cext_sensor, double* cext_total, int32_t* iters, double* rel_resid);

// Device bytes the solve phase allocates (GMRES state and operator workspaces) for one batch of
// B wavelengths on a geometry of N panels and S surfaces.
int64_t solve_bytes(int64_t N, int S, int B, const lspr_op_params& op,
                    const lspr_gmres_params& gm);
// Upper bound of the matrix-core tile store kept for a geometry of N panels in the given
// precision mode (larger stores fall back to the on-the-fly kernel).
int64_t tile_cap_bytes(int64_t N, const lspr_op_params& op);
// Upper bound of the device bytes one request holds at its peak (set-up, tiles, solve).
int64_t request_footprint(int64_t N, int S, int n_lambda, const lspr_op_params& op,
                          const lspr_gmres_params& gm);

}  // namespace lspr
