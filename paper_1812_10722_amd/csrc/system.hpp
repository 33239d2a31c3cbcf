// System-level entry points (system.hip, gmres.hip, post.hip).
#pragma once

#include "internal.hpp"

namespace lspr {

struct EpsSet {
    std::vector<double> em_re, em_im;  // [B]
    std::vector<double> es_re, es_im;  // [B][S]
};

// ratio[b][s] = eps_surface[b][s] / eps_medium[b] on the host ([B][S]), and on the device
// (grow-only buffer; with point charges also 1 / eps_s for the right-hand side).
std::vector<double2> ratio_values(const Geometry& g, const EpsSet& eps, int B);
void upload_ratios(Geometry& g, const EpsSet& eps, int B, DevBuf<double2>& d, hipStream_t s);
// Bytes of scratch one lspr_apply batch of B columns needs in precision prec (ratios, the
// sorted copies of x and y, packed densities, raw sums, moments, P2M partial sums), counted in
// the arena's 256-byte pieces.
size_t apply_scratch_bytes(const Geometry& g, int B, int prec);

// y[col] = A(col) x[col] for nslot columns; col = d_cols[slot] (or slot when d_cols is null),
// with far-field products in precision prec (LSPR_FP32 or LSPR_FP64); with precond,
// y[col] = A(col) M(col)^-1 x[col] (M: the 2x2 self-panel blocks, precond.hpp).
// Vectors are complex [*][2N] in sorted panel order with the given strides (in elements).
void system_apply(Geometry& g, int prec, int nslot, const double2* ratio_d, const double2* x,
                  int64_t x_stride, double2* y, int64_t y_stride, const int32_t* d_cols,
                  hipStream_t s, bool precond = false);

// Point charges (host arrays: positions [n_q][3], values, surfaces); n_q = 0 removes them.
void set_charges(Geometry& g, int n_q, const double* pos, const double* q, const int32_t* sid,
                 hipStream_t s);

// b[col] for columns 0..ncolumn-1 (sorted order, stride b_stride); with charges, the
// permittivities of the batch must have been uploaded (upload_ratios) first.
void system_rhs(Geometry& g, int ncolumn, const double2* ratio_d, const double* e_field,
                double2* b, int64_t b_stride, hipStream_t s);

struct SolveResult {
    std::vector<int32_t> iters;
    std::vector<double> rel_resid;
    bool all_converged = true;
};

// Batched GMRES for columns 0..B-1 with far-field products in precision prec; b_in holds the
// right-hand sides [B][2N] (sorted order), or is null for the system's own (e_field);
// x_out receives the solutions [B][2N] (sorted order).
SolveResult gmres_solve(Geometry& g, int prec, int B, const double2* ratio_d,
                        const double* e_field, const lspr_gmres_params& gm, const double2* b_in,
                        double2* x_out, hipStream_t s);

// Iterative refinement with FP32 inner solves and FP64 residuals (LSPR_FP32_REFINE64).
SolveResult refine_solve(Geometry& g, int B, const double2* ratio_d, const double* e_field,
                         const lspr_gmres_params& gm, double2* x_out, hipStream_t s);

// Dipole moments q = p / eps_m (sensor only and total) for each column: host [B][2][3] complex.
void dipole_moments(Geometry& g, int B, const double2* ratio_d, const double* e_field,
                    const double2* x, std::vector<double>& q, hipStream_t s);

// Scatter sorted-order solutions to the caller's order: phi [B][N], dphi [B][N] (device).
void unpermute(Geometry& g, int B, const double2* x, double2* phi, double2* dphi, hipStream_t s);
// Gather caller-order vectors [B][2N] into sorted order, and back.
void to_sorted(Geometry& g, int B, const double2* in, double2* out, hipStream_t s);
void from_sorted(Geometry& g, int B, const double2* in, double2* out, hipStream_t s);

}  // namespace lspr
