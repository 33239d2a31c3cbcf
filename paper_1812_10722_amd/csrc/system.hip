// The complex block systems of Eq. matrix_lspr / Eq. matrix_multi on top of the real layer
// operators, their right-hand side, a batched complex GMRES with the Arnoldi process on the
// device (section "Code modifications and added features": GMRES for complex numbers), and
// the dipole moment / extinction cross-section post-processing.
//
// Unknowns per wavelength, in sorted panel order: phi (N values) then psi = dphi/dn on the
// interior side (N values).  For target panel i of surface t and eps ratios r_s = eps_s/eps_m:
//   interior row:  phi_i/2 + sum_{j in t} K_ij phi_j - sum_{j in t} V_ij psi_j = 0
//   exterior row:  phi_i/2 - sum_j K_ij phi_j + sum_j r_s(j) V_ij psi_j
//                      = sum_j (1 - r_s(j)) V_ij g_j,     g = dphi_inc/dn = -E . n.
// The V columns carry sigma_j = r_s(j) psi_j, so the own-surface V sum divided by r_t gives
// the interior row's V psi term.
#include <cmath>
#include <cstdio>

#include "operator.hpp"
#include "precond.hpp"
#include "profile.hpp"
#include "system.hpp"

namespace lspr {

namespace {

constexpr int TPB = 256;
constexpr double INV_4PI = 0.07957747154594767;  // 1 / (4 pi)

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

// Unknowns (phi, psi) of panel i of column col: x itself, or M^-1 x when vself is given.
__device__ __forceinline__ void unknowns(const double2* xc, int N, int i, double2 r,
                                         const double* vself, double2& phi, double2& psi) {
    phi = xc[i];
    psi = xc[N + i];
    if (vself != nullptr) block_jacobi(phi, psi, r, vself[i] * INV_4PI, phi, psi);
}

// x (complex, [col][2N] sorted order) -> packed real columns dens [N][2 pad]:
// K columns 2s, 2s+1 = Re, Im phi; V columns pad + 2s, pad + 2s + 1 = Re, Im sigma.
// Block = pp consecutive panels, all columns: (slot, panel) pairs with the panel fastest read
// the vectors along the panels; the rows are assembled in LDS (row stride 2 pad + 1 elements,
// so that consecutive panels fall in different banks) and written whole.
template <class T>
__global__ void __launch_bounds__(TPB) k_pack(const double2* __restrict__ x, int64_t x_stride,
                                              const int32_t* __restrict__ cols, int nslot, int N,
                                              const double2* __restrict__ ratio, int S,
                                              const int32_t* __restrict__ surf,
                                              const double* __restrict__ vself, int pad, int pp,
                                              T* __restrict__ dens) {
    extern __shared__ double pack_sh[];
    T* tile = reinterpret_cast<T*>(pack_sh);
    const int ncols = 2 * pad, ld = ncols + 1;
    const int i0 = blockIdx.x * pp, np = min(pp, N - i0);
    for (int u = threadIdx.x; u < (pad / 2) * pp; u += TPB) {
        const int p = u % pp, slot = u / pp, i = i0 + p;
        T a = T(0), b = T(0), c = T(0), d = T(0);
        if (p < np && slot < nslot) {
            const int col = cols ? cols[slot] : slot;
            const double2 r = ratio[col * S + surf[i]];
            double2 phi, psi;
            unknowns(x + col * x_stride, N, i, r, vself, phi, psi);
            const double2 sig = cmul(r, psi);
            a = static_cast<T>(phi.x);
            b = static_cast<T>(phi.y);
            c = static_cast<T>(sig.x);
            d = static_cast<T>(sig.y);
        }
        T* row = tile + p * ld;
        row[2 * slot] = a;
        row[2 * slot + 1] = b;
        row[pad + 2 * slot] = c;
        row[pad + 2 * slot + 1] = d;
    }
    __syncthreads();
    T* dst = dens + static_cast<size_t>(i0) * ncols;
    for (int e = threadIdx.x; e < np * ncols; e += TPB) dst[e] = tile[(e / ncols) * ld + e % ncols];
}

// One output pair (interior, exterior row) of column `slot` at panel i, from its rows of raw
// sums (rs: own surface, ra: all surfaces).
__device__ __forceinline__ void combine_one(const double2* __restrict__ x, int64_t x_stride,
                                            double2* __restrict__ y, int64_t y_stride,
                                            const int32_t* __restrict__ cols, int slot, int N,
                                            int i, const double2* __restrict__ ratio, int S,
                                            const int32_t* __restrict__ surf,
                                            const double* __restrict__ vself, int pad,
                                            const double* rs, const double* ra) {
    const int col = cols ? cols[slot] : slot;
    double2 phi, psi;
    unknowns(x + col * x_stride, N, i, ratio[col * S + surf[i]], vself, phi, psi);
    const double2 k_all = make_double2(ra[2 * slot] * INV_4PI, ra[2 * slot + 1] * INV_4PI);
    const double2 v_all = make_double2(ra[pad + 2 * slot] * INV_4PI, ra[pad + 2 * slot + 1] * INV_4PI);
    const double2 k_own = make_double2(rs[2 * slot] * INV_4PI, rs[2 * slot + 1] * INV_4PI);
    const double2 v_own = make_double2(rs[pad + 2 * slot] * INV_4PI, rs[pad + 2 * slot + 1] * INV_4PI);
    const double2 r = ratio[col * S + surf[i]];
    const double den = r.x * r.x + r.y * r.y;
    const double2 rinv = make_double2(r.x / den, -r.y / den);
    const double2 vpsi = cmul(rinv, v_own);
    double2* yc = y + col * y_stride;
    yc[i] = make_double2(0.5 * phi.x + k_own.x - vpsi.x, 0.5 * phi.y + k_own.y - vpsi.y);
    yc[N + i] = make_double2(0.5 * phi.x - k_all.x + v_all.x, 0.5 * phi.y - k_all.y + v_all.y);
}

// Rows of Eq. matrix_multi from the raw sums (no 1/4pi yet).  Block = pp consecutive panels:
// their rows of raw sums are read whole into LDS (row stride 2 pad + 1), then (slot, panel)
// pairs with the panel fastest read x and write y along the panels.
__global__ void __launch_bounds__(TPB) k_combine(const double2* __restrict__ x, int64_t x_stride,
                                                 double2* __restrict__ y, int64_t y_stride,
                                                 const int32_t* __restrict__ cols, int nslot,
                                                 int N, const double2* __restrict__ ratio, int S,
                                                 const int32_t* __restrict__ surf,
                                                 const double* __restrict__ vself, int pad,
                                                 int pp, const double* __restrict__ out_self,
                                                 const double* __restrict__ out_all) {
    extern __shared__ double comb_sh[];
    const int ncols = 2 * pad, ld = ncols + 1;
    const int i0 = blockIdx.x * pp, np = min(pp, N - i0);
    double* ta = comb_sh;
    double* ts = out_self ? comb_sh + pp * ld : comb_sh;
    for (int e = threadIdx.x; e < np * ncols; e += TPB) {
        const int p = e / ncols, c = e % ncols;
        ta[p * ld + c] = out_all[static_cast<size_t>(i0) * ncols + e];
        if (out_self) ts[p * ld + c] = out_self[static_cast<size_t>(i0) * ncols + e];
    }
    __syncthreads();
    for (int u = threadIdx.x; u < nslot * pp; u += TPB) {
        const int p = u % pp, slot = u / pp, i = i0 + p;
        if (p < np) combine_one(x, x_stride, y, y_stride, cols, slot, N, i, ratio, S, surf,
                                vself, pad, ts + p * ld, ta + p * ld);
    }
}

// b = [cu / eps_s; sum_s (1 - r_s) sum_d E_d u[s][d] / 4pi] per column (cu: the point charges'
// potential times eps_s on the interior rows of their surface, or null)
__global__ void k_rhs(const double* __restrict__ u, int S, int N, int ncolumn,
                      const double2* __restrict__ ratio, double e0, double e1, double e2,
                      const double* __restrict__ cu, const double2* __restrict__ inv_eps,
                      const int32_t* __restrict__ surf, double2* __restrict__ b,
                      int64_t b_stride) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(N) * ncolumn) return;
    const int col = static_cast<int>(t / N), i = static_cast<int>(t % N);
    double2 acc = make_double2(0.0, 0.0);
    for (int s = 0; s < S; ++s) {
        const double us = (e0 * u[(3 * s) * N + i] + e1 * u[(3 * s + 1) * N + i] +
                           e2 * u[(3 * s + 2) * N + i]) * INV_4PI;
        const double2 r = ratio[col * S + s];
        acc.x += (1.0 - r.x) * us;
        acc.y += -r.y * us;
    }
    double2 in = make_double2(0.0, 0.0);
    if (cu != nullptr) {
        const double2 ie = inv_eps[col * S + surf[i]];
        in = make_double2(cu[i] * ie.x, cu[i] * ie.y);
    }
    b[col * b_stride + i] = in;
    b[col * b_stride + N + i] = acc;
}

// charge_u[i] = sum over the charges of panel i's surface (off[s] .. off[s + 1]) of
// q_k / (4 pi |c_i - r_k|), in order
__global__ void k_charge_u(const double* __restrict__ cen, const int32_t* __restrict__ surf,
                           int N, const double* __restrict__ pos, const double* __restrict__ q,
                           const int32_t* __restrict__ off, double* __restrict__ cu) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int s = surf[i];
    double acc = 0.0;
    for (int k = off[s]; k < off[s + 1]; ++k) {
        const double dx = cen[3 * i] - pos[3 * k], dy = cen[3 * i + 1] - pos[3 * k + 1],
                     dz = cen[3 * i + 2] - pos[3 * k + 2];
        acc += q[k] / sqrt(dx * dx + dy * dy + dz * dz);
    }
    cu[i] = acc * INV_4PI;
}

// RHS geometry columns: V column 3s + d holds -n_d on surface s, zero elsewhere.
template <class T>
__global__ void k_rhs_dens(const double* __restrict__ nrm, const int32_t* __restrict__ surf,
                           int N, int S, int pad, T* __restrict__ dens) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(N) * 2 * pad) return;
    const int i = static_cast<int>(t / (2 * pad)), c = static_cast<int>(t % (2 * pad));
    T v = T(0);
    if (c >= pad && c - pad < 3 * S) {
        const int s = (c - pad) / 3, d = (c - pad) % 3;
        if (surf[i] == s) v = static_cast<T>(-nrm[3 * i + d]);
    }
    dens[t] = v;
}

__global__ void k_rhs_extract(const double* __restrict__ out, int N, int S, int pad,
                              double* __restrict__ u) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(N) * 3 * S) return;
    const int k = static_cast<int>(t / N), i = static_cast<int>(t % N);
    u[t] = out[static_cast<size_t>(i) * 2 * pad + pad + k];
}

}  // namespace

void precompute_rhs(Geometry& g) {
    hipStream_t s = g.stream;
    // in FP64 whenever the geometry runs FP64 products
    const Cols c = make_cols(g, 3 * g.S, g.need64 ? LSPR_FP64 : LSPR_FP32);
    const size_t nd = static_cast<size_t>(g.N) * 2 * c.pad;
    const size_t esz = c.prec == LSPR_FP32 ? 4 : 8;
    DevBuf<uint8_t> dens(nd * esz);
    DevBuf<double> oa(nd), os(g.S > 1 ? nd : 0);
    const int64_t tot = static_cast<int64_t>(nd);
    if (c.prec == LSPR_FP32)
        hipLaunchKernelGGL(k_rhs_dens<float>, dim3((tot + TPB - 1) / TPB), dim3(TPB), 0, s,
                           g.nrm.p, g.surf.p, g.N, g.S, c.pad, reinterpret_cast<float*>(dens.p));
    else
        hipLaunchKernelGGL(k_rhs_dens<double>, dim3((tot + TPB - 1) / TPB), dim3(TPB), 0, s,
                           g.nrm.p, g.surf.p, g.N, g.S, c.pad, reinterpret_cast<double*>(dens.p));
    LSPR_HIP(hipGetLastError());
    apply_raw(g, c, dens.p, os.p, oa.p, s);
    g.rhs_u.alloc(static_cast<size_t>(3) * g.S * g.N);
    const int64_t nu = static_cast<int64_t>(3) * g.S * g.N;
    hipLaunchKernelGGL(k_rhs_extract, dim3((nu + TPB - 1) / TPB), dim3(TPB), 0, s, oa.p, g.N,
                       g.S, c.pad, g.rhs_u.p);
    LSPR_HIP(hipGetLastError());
    LSPR_HIP(hipStreamSynchronize(s));
}

std::vector<double2> ratio_values(const Geometry& g, const EpsSet& eps, int B) {
    std::vector<double2> h(static_cast<size_t>(B) * g.S);
    for (int b = 0; b < B; ++b) {
        const double mr = eps.em_re[b], mi = eps.em_im[b];
        const double den = mr * mr + mi * mi;
        LSPR_REQUIRE(den > 0.0, LSPR_E_INVALID, "eps_medium must be nonzero");
        for (int k = 0; k < g.S; ++k) {
            const double sr = eps.es_re[b * g.S + k], si = eps.es_im[b * g.S + k];
            LSPR_REQUIRE(sr * sr + si * si > 1e-24 * den, LSPR_E_INVALID,
                         "eps_surface must be nonzero");
            h[b * g.S + k] = make_double2((sr * mr + si * mi) / den, (si * mr - sr * mi) / den);
        }
    }
    return h;
}

void upload_ratios(Geometry& g, const EpsSet& eps, int B, DevBuf<double2>& d, hipStream_t s) {
    const std::vector<double2> h = ratio_values(g, eps, B);
    d.reserve(h.size());
    LSPR_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(double2), hipMemcpyHostToDevice, s));
    if (g.charge_u.p != nullptr) {  // 1 / eps_s for the charges' right-hand side
        std::vector<double2> ie(static_cast<size_t>(B) * g.S);
        for (size_t k = 0; k < ie.size(); ++k) {
            const double sr = eps.es_re[k], si = eps.es_im[k], dd = sr * sr + si * si;
            ie[k] = make_double2(sr / dd, -si / dd);
        }
        g.ws_inv_eps.reserve(ie.size());
        LSPR_HIP(hipMemcpyAsync(g.ws_inv_eps.p, ie.data(), ie.size() * sizeof(double2),
                                hipMemcpyHostToDevice, s));
        LSPR_HIP(hipStreamSynchronize(s));  // ie is local
    }
    LSPR_HIP(hipStreamSynchronize(s));  // h is local
}

void set_charges(Geometry& g, int n_q, const double* pos, const double* q, const int32_t* sid,
                 hipStream_t s) {
    g.charge_u.release();
    if (n_q == 0) return;
    std::vector<int32_t> off(g.S + 1, 0);
    for (int k = 0; k < n_q; ++k) {
        LSPR_REQUIRE(sid[k] >= 0 && sid[k] < g.S, LSPR_E_INVALID, "charge surface out of range");
        LSPR_REQUIRE(std::isfinite(pos[3 * k]) && std::isfinite(pos[3 * k + 1]) &&
                         std::isfinite(pos[3 * k + 2]) && std::isfinite(q[k]),
                     LSPR_E_INVALID, "charges must be finite");
        ++off[sid[k] + 1];
    }
    for (int t = 0; t < g.S; ++t) off[t + 1] += off[t];
    std::vector<double> p_s(3 * static_cast<size_t>(n_q)), q_s(n_q);
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int k = 0; k < n_q; ++k) {  // grouped by surface, input order kept within a surface
        const int at = fill[sid[k]]++;
        for (int d = 0; d < 3; ++d) p_s[3 * at + d] = pos[3 * k + d];
        q_s[at] = q[k];
    }
    DevBuf<double> pd(p_s.size()), qd(q_s.size());
    DevBuf<int32_t> od(off.size());
    copy_sync(pd.p, p_s.data(), p_s.size() * 8, hipMemcpyHostToDevice, s);
    copy_sync(qd.p, q_s.data(), q_s.size() * 8, hipMemcpyHostToDevice, s);
    copy_sync(od.p, off.data(), off.size() * 4, hipMemcpyHostToDevice, s);
    g.charge_u.alloc(g.N);
    hipLaunchKernelGGL(k_charge_u, dim3((g.N + TPB - 1) / TPB), dim3(TPB), 0, s, g.cen.p,
                       g.surf.p, g.N, pd.p, qd.p, od.p, g.charge_u.p);
    LSPR_HIP(hipGetLastError());
    LSPR_HIP(hipStreamSynchronize(s));
}

// y[col] = A(eps[col]) x[col] for the nslot columns listed in d_cols (or 0..nslot-1).
void system_apply(Geometry& g, int prec, int nslot, const double2* ratio_d, const double2* x,
                  int64_t x_stride, double2* y, int64_t y_stride, const int32_t* d_cols,
                  hipStream_t s, bool precond) {
    const double* vs = precond ? g.vself.p : nullptr;
    const Cols c = make_cols(g, 2 * nslot, prec);
    const size_t nd = static_cast<size_t>(g.N) * 2 * c.pad;
    const size_t esz = c.prec == LSPR_FP32 ? 4 : 8;
    prof::Scope sc("matvec", s, 0.0, 0.0);
    uint8_t* dens = workspace(g, g.ws_dens, nd * esz);
    double* oa = reinterpret_cast<double*>(
        workspace(g, g.ws_out, nd * sizeof(double) * (g.S > 1 ? 2 : 1)));
    double* os = g.S > 1 ? oa + nd : nullptr;
    // panels per block of the packing and combining kernels: their LDS rows within 48 KB
    auto panels_per_block = [&](size_t row_bytes) {
        int pp = 32;
        while (pp > 1 && static_cast<size_t>(pp) * row_bytes > 48 * 1024) pp /= 2;
        return pp;
    };
    const size_t ld = static_cast<size_t>(2 * c.pad + 1);
    const int ppk = panels_per_block(ld * esz);
    const int nbk = (g.N + ppk - 1) / ppk;
    if (c.prec == LSPR_FP32)
        hipLaunchKernelGGL(k_pack<float>, dim3(nbk), dim3(TPB), ppk * ld * esz, s, x, x_stride,
                           d_cols, nslot, g.N, ratio_d, g.S, g.surf.p, vs, c.pad, ppk,
                           reinterpret_cast<float*>(dens));
    else
        hipLaunchKernelGGL(k_pack<double>, dim3(nbk), dim3(TPB), ppk * ld * esz, s, x, x_stride,
                           d_cols, nslot, g.N, ratio_d, g.S, g.surf.p, vs, c.pad, ppk,
                           reinterpret_cast<double*>(dens));
    LSPR_HIP(hipGetLastError());
    apply_raw(g, c, dens, os, oa, s);
    const size_t crow = ld * sizeof(double) * (os ? 2 : 1);
    const int ppc = panels_per_block(crow);
    hipLaunchKernelGGL(k_combine, dim3((g.N + ppc - 1) / ppc), dim3(TPB), ppc * crow, s, x,
                       x_stride, y, y_stride, d_cols, nslot, g.N, ratio_d, g.S, g.surf.p, vs,
                       c.pad, ppc, os, oa);
    LSPR_HIP(hipGetLastError());
}

void system_rhs(Geometry& g, int ncolumn, const double2* ratio_d, const double* e_field,
                double2* b, int64_t b_stride, hipStream_t s) {
    const int64_t t = static_cast<int64_t>(g.N) * ncolumn;
    const bool q = g.charge_u.p != nullptr;
    LSPR_REQUIRE(!q || g.ws_inv_eps.n >= static_cast<size_t>(ncolumn) * g.S, LSPR_E_INVALID,
                 "permittivities of the batch not uploaded");
    hipLaunchKernelGGL(k_rhs, dim3((t + TPB - 1) / TPB), dim3(TPB), 0, s, g.rhs_u.p, g.S, g.N,
                       ncolumn, ratio_d, e_field[0], e_field[1], e_field[2],
                       q ? g.charge_u.p : nullptr, q ? g.ws_inv_eps.p : nullptr, g.surf.p, b,
                       b_stride);
    LSPR_HIP(hipGetLastError());
}

}  // namespace lspr
