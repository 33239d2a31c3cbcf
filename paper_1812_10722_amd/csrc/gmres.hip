// Batched restarted GMRES in complex FP64 (section "Code modifications and added features":
// the solver accepts complex numbers; the paper fixes only tolerances, Tables 2 and 5).
//
// Every wavelength has its own Krylov space; all running wavelengths share each block
// matrix-vector product.  The Arnoldi process runs on the device: classical Gram-Schmidt with
// one re-orthogonalisation pass (two dot/update sweeps), the norm, the Givens rotations and
// the residual estimate |g_{j+1}|.  The host only launches kernels and reads one residual
// estimate per wavelength per iteration to retire converged wavelengths, which then leave the
// matrix-vector product.  x0 = 0; a wavelength stops when ||b - A x|| <= tol ||b||, checked
// on the true residual at each restart.  Optional right block-Jacobi preconditioning with the
// 2x2 self-panel blocks (K_ii = 0 on flat panels) does not change the solution.
#include <algorithm>
#include <cmath>

#include "profile.hpp"
#include "system.hpp"

namespace lspr {

namespace {

constexpr int GT = 256;
constexpr int GE = 8;
constexpr int GSLICE = GT * GE;
constexpr double INV_4PI = 0.07957747154594767;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconjmul(double2 a, double2 b) {
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// part[(slot * m1 + i) * nblk + blk] = sum over the block's slice of conj(V_i) . w, i <= j
__global__ void __launch_bounds__(GT) k_dots(const double2* __restrict__ V, int m1,
                                             int64_t nvec, int j, const double2* __restrict__ w,
                                             const int32_t* __restrict__ cols,
                                             double2* __restrict__ part, int nblk) {
    extern __shared__ double2 red[];  // [GT/64][j+1]
    const int slot = blockIdx.y, col = cols[slot];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * GSLICE;
    const double2* wc = w + col * nvec;
    double2 wl[GE];
#pragma unroll
    for (int e = 0; e < GE; ++e) {
        const int64_t n = base + e * GT + threadIdx.x;
        wl[e] = n < nvec ? wc[n] : make_double2(0.0, 0.0);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = 0; i <= j; ++i) {
        const double2* vi = V + (static_cast<int64_t>(col) * m1 + i) * nvec;
        double ar = 0.0, ai = 0.0;
#pragma unroll
        for (int e = 0; e < GE; ++e) {
            const int64_t n = base + e * GT + threadIdx.x;
            if (n < nvec) {
                const double2 p = cconjmul(vi[n], wl[e]);
                ar += p.x;
                ai += p.y;
            }
        }
        ar = wave_sum(ar);
        ai = wave_sum(ai);
        if (lane == 0) red[wave * (j + 1) + i] = make_double2(ar, ai);
    }
    __syncthreads();
    for (int i = threadIdx.x; i <= j; i += GT) {
        double2 s = make_double2(0.0, 0.0);
        for (int q = 0; q < GT / 64; ++q) {
            s.x += red[q * (j + 1) + i].x;
            s.y += red[q * (j + 1) + i].y;
        }
        part[(static_cast<int64_t>(slot) * m1 + i) * nblk + blockIdx.x] = s;
    }
}

// hpass[col][i] = sum_blk part; hcol[col][i] (+)= hpass
__global__ void k_dots_final(const double2* __restrict__ part, int nblk, int m1, int j,
                             const int32_t* __restrict__ cols, int nslot,
                             double2* __restrict__ hpass, double2* __restrict__ hcol, int accum) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nslot * (j + 1)) return;
    const int slot = t / (j + 1), i = t % (j + 1);
    const int col = cols[slot];
    double2 s = make_double2(0.0, 0.0);
    const double2* p = part + (static_cast<int64_t>(slot) * m1 + i) * nblk;
    for (int b = 0; b < nblk; ++b) {
        s.x += p[b].x;
        s.y += p[b].y;
    }
    hpass[col * m1 + i] = s;
    if (accum) {
        hcol[col * m1 + i].x += s.x;
        hcol[col * m1 + i].y += s.y;
    } else {
        hcol[col * m1 + i] = s;
    }
}

// w -= sum_{i <= j} V_i hpass_i
__global__ void __launch_bounds__(GT) k_update(const double2* __restrict__ V, int m1,
                                               int64_t nvec, int j, double2* __restrict__ w,
                                               const int32_t* __restrict__ cols,
                                               const double2* __restrict__ hpass) {
    const int col = cols[blockIdx.y];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * GSLICE;
    double2* wc = w + col * nvec;
#pragma unroll
    for (int e = 0; e < GE; ++e) {
        const int64_t n = base + e * GT + threadIdx.x;
        if (n >= nvec) continue;
        double2 a = wc[n];
        for (int i = 0; i <= j; ++i) {
            const double2 p = cmul(V[(static_cast<int64_t>(col) * m1 + i) * nvec + n], hpass[col * m1 + i]);
            a.x -= p.x;
            a.y -= p.y;
        }
        wc[n] = a;
    }
}

// part2[slot * nblk + blk] = sum |w|^2 over the slice
__global__ void __launch_bounds__(GT) k_norm_part(const double2* __restrict__ w, int64_t nvec,
                                                  int64_t stride, const int32_t* __restrict__ cols,
                                                  double* __restrict__ part2, int nblk) {
    __shared__ double red[GT / 64];
    const int col = cols[blockIdx.y];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * GSLICE;
    const double2* wc = w + col * stride;
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < GE; ++e) {
        const int64_t n = base + e * GT + threadIdx.x;
        if (n < nvec) s += wc[n].x * wc[n].x + wc[n].y * wc[n].y;
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int q = 0; q < GT / 64; ++q) t += red[q];
        part2[static_cast<int64_t>(blockIdx.y) * nblk + blockIdx.x] = t;
    }
}

// Finishes Arnoldi step j for each running column: h_{j+1,j} = ||w||, previous rotations on
// column j, new rotation zeroing h_{j+1,j}, g update, residual estimate, 1/||w||.
__global__ void k_arnoldi_finish(const double* __restrict__ part2, int nblk,
                                 const int32_t* __restrict__ cols, int nslot, int m, int j,
                                 double2* __restrict__ hcol, double2* __restrict__ H,
                                 double2* __restrict__ cs, double2* __restrict__ sn,
                                 double2* __restrict__ gv, double* __restrict__ est,
                                 double* __restrict__ inv_norm) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= nslot) return;
    const int col = cols[slot];
    const int m1 = m + 1;
    double ss = 0.0;
    for (int b = 0; b < nblk; ++b) ss += part2[static_cast<int64_t>(slot) * nblk + b];
    const double nrm = sqrt(ss);
    double2* h = hcol + col * m1;
    h[j + 1] = make_double2(nrm, 0.0);
    double2* c = cs + col * m;
    double2* s = sn + col * m;
    for (int i = 0; i < j; ++i) {  // [x, y] -> [conj(c) x + conj(s) y, -s x + c y]
        const double2 hi = h[i], hn = h[i + 1];
        const double2 a = cconjmul(c[i], hi), bq = cconjmul(s[i], hn);
        const double2 d = cmul(s[i], hi), e = cmul(c[i], hn);
        h[i] = make_double2(a.x + bq.x, a.y + bq.y);
        h[i + 1] = make_double2(e.x - d.x, e.y - d.y);
    }
    const double2 a = h[j], bq = h[j + 1];
    const double den = sqrt(a.x * a.x + a.y * a.y + bq.x * bq.x + bq.y * bq.y);
    double2 cj = make_double2(1.0, 0.0), sj = make_double2(0.0, 0.0);
    if (den > 0.0) {
        cj = make_double2(a.x / den, a.y / den);
        sj = make_double2(bq.x / den, bq.y / den);
    }
    c[j] = cj;
    s[j] = sj;
    h[j] = make_double2(den, 0.0);
    h[j + 1] = make_double2(0.0, 0.0);
    double2* g = gv + col * m1;
    const double2 gj = g[j];
    const double2 t = cmul(sj, gj);
    g[j + 1] = make_double2(-t.x, -t.y);
    g[j] = cconjmul(cj, gj);
    for (int i = 0; i <= j + 1; ++i) H[(static_cast<int64_t>(col) * m + j) * m1 + i] = h[i];
    est[col] = sqrt(g[j + 1].x * g[j + 1].x + g[j + 1].y * g[j + 1].y);
    inv_norm[col] = nrm > 0.0 ? 1.0 / nrm : 0.0;
}

// dst_col = src_col * scale[col]
// (src and dst may be the same vectors: the scaling is element-wise)
__global__ void __launch_bounds__(GT) k_scale(const double2* src, int64_t src_stride,
                                              double2* dst, int64_t dst_stride,
                                              int64_t nvec, const int32_t* __restrict__ cols,
                                              const double* __restrict__ scale) {
    const int col = cols[blockIdx.y];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * GSLICE;
    const double f = scale[col];
#pragma unroll
    for (int e = 0; e < GE; ++e) {
        const int64_t n = base + e * GT + threadIdx.x;
        if (n < nvec) {
            const double2 v = src[col * src_stride + n];
            dst[col * dst_stride + n] = make_double2(v.x * f, v.y * f);
        }
    }
}

// y = R^{-1} g with R the jn x jn upper triangle of the rotated Hessenberg matrix.
__global__ void k_backsolve(const double2* __restrict__ H, const double2* __restrict__ gv,
                            const int32_t* __restrict__ jn, const int32_t* __restrict__ cols,
                            int nslot, int m, double2* __restrict__ y) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= nslot) return;
    const int col = cols[slot];
    const int n = jn[col], m1 = m + 1;
    const double2* Hc = H + static_cast<int64_t>(col) * m * m1;  // column k at Hc + k*m1
    double2* yc = y + col * m;
    for (int k = n - 1; k >= 0; --k) {
        double2 r = gv[col * m1 + k];
        for (int l = k + 1; l < n; ++l) {
            const double2 p = cmul(Hc[l * m1 + k], yc[l]);
            r.x -= p.x;
            r.y -= p.y;
        }
        const double2 d = Hc[k * m1 + k];
        yc[k] = (d.x == 0.0 && d.y == 0.0) ? make_double2(0.0, 0.0) : cdiv(r, d);
    }
}

// u_col = sum_{k < jn} y_k V_k
__global__ void __launch_bounds__(GT) k_basis_combine(const double2* __restrict__ V, int m1,
                                                      int64_t nvec, const double2* __restrict__ y,
                                                      int m, const int32_t* __restrict__ jn,
                                                      const int32_t* __restrict__ cols,
                                                      double2* __restrict__ u) {
    const int col = cols[blockIdx.y];
    const int n = jn[col];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * GSLICE;
#pragma unroll
    for (int e = 0; e < GE; ++e) {
        const int64_t q = base + e * GT + threadIdx.x;
        if (q >= nvec) continue;
        double2 a = make_double2(0.0, 0.0);
        for (int k = 0; k < n; ++k) {
            const double2 p = cmul(V[(static_cast<int64_t>(col) * m1 + k) * nvec + q], y[col * m + k]);
            a.x += p.x;
            a.y += p.y;
        }
        u[col * nvec + q] = a;
    }
}

// out_col (+)= M^{-1} in_col with M_i = [[1/2, -v_i], [1/2, r v_i]] (v_i = V_ii)
__global__ void k_precond(const double2* __restrict__ in, int64_t in_stride,
                          double2* __restrict__ out, int64_t out_stride, int N,
                          const int32_t* __restrict__ cols, int nslot,
                          const double2* __restrict__ ratio, int S,
                          const int32_t* __restrict__ surf, const double* __restrict__ vself,
                          int add) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(N) * nslot) return;
    const int slot = static_cast<int>(t / N), i = static_cast<int>(t % N);
    const int col = cols[slot];
    const double2 a = in[col * in_stride + i], b = in[col * in_stride + N + i];
    const double2 r = ratio[col * S + surf[i]];
    const double v = vself[i] * INV_4PI;
    const double2 onep = make_double2(1.0 + r.x, r.y);
    // phi = 2 (r a + b) / (1 + r);  psi = (b - a) / (v (1 + r))
    const double2 ra = cmul(r, a);
    double2 phi = cdiv(make_double2(2.0 * (ra.x + b.x), 2.0 * (ra.y + b.y)), onep);
    double2 psi = cdiv(make_double2((b.x - a.x) / v, (b.y - a.y) / v), onep);
    double2* o = out + col * out_stride;
    if (add) {
        o[i].x += phi.x;
        o[i].y += phi.y;
        o[N + i].x += psi.x;
        o[N + i].y += psi.y;
    } else {
        o[i] = phi;
        o[N + i] = psi;
    }
}

// dst_col (+)= src_col; r_col = b_col - w_col
__global__ void __launch_bounds__(GT) k_axpy(const double2* __restrict__ a, double2* __restrict__ d,
                                             int64_t nvec, const int32_t* __restrict__ cols) {
    const int col = cols[blockIdx.y];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * GSLICE;
#pragma unroll
    for (int e = 0; e < GE; ++e) {
        const int64_t n = base + e * GT + threadIdx.x;
        if (n < nvec) {
            d[col * nvec + n].x += a[col * nvec + n].x;
            d[col * nvec + n].y += a[col * nvec + n].y;
        }
    }
}

__global__ void __launch_bounds__(GT) k_resid(const double2* __restrict__ b,
                                              const double2* __restrict__ w,
                                              double2* __restrict__ r, int64_t r_stride,
                                              int64_t nvec, const int32_t* __restrict__ cols) {
    const int col = cols[blockIdx.y];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * GSLICE;
#pragma unroll
    for (int e = 0; e < GE; ++e) {
        const int64_t n = base + e * GT + threadIdx.x;
        if (n < nvec)
            r[col * r_stride + n] = make_double2(b[col * nvec + n].x - w[col * nvec + n].x,
                                                 b[col * nvec + n].y - w[col * nvec + n].y);
    }
}

__global__ void k_set_g(double2* __restrict__ gv, int m1, const int32_t* __restrict__ cols,
                        int nslot, const double* __restrict__ beta) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nslot * m1) return;
    const int slot = t / m1, i = t % m1;
    const int col = cols[slot];
    gv[col * m1 + i] = make_double2(i == 0 ? beta[col] : 0.0, 0.0);
}

__global__ void k_norm_final(const double* __restrict__ part2, int nblk,
                             const int32_t* __restrict__ cols, int nslot,
                             double* __restrict__ nrm, double* __restrict__ inv) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= nslot) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part2[static_cast<int64_t>(slot) * nblk + b];
    const int col = cols[slot];
    nrm[col] = sqrt(s);
    inv[col] = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
}

int blocks_for(int64_t nvec) { return static_cast<int>((nvec + GSLICE - 1) / GSLICE); }

}  // namespace

SolveResult gmres_solve(Geometry& g, int prec, int B, const double2* ratio_d,
                        const double* e_field, const lspr_gmres_params& gm, const double2* b_in,
                        double2* x, hipStream_t s) {
    const int m = gm.restart, m1 = m + 1;
    const int64_t nvec = 2 * static_cast<int64_t>(g.N);
    const int nblk = blocks_for(nvec);
    const bool pre = gm.precond != 0;
    DevBuf<double2> V(static_cast<size_t>(B) * m1 * nvec), w(B * nvec), bvec(B * nvec);
    DevBuf<double2> z(pre ? B * nvec : 0);
    DevBuf<double2> hcol(B * m1), hpass(B * m1), H(static_cast<size_t>(B) * m * m1);
    DevBuf<double2> cs(B * m), sn(B * m), gv(B * m1), y(B * m);
    DevBuf<double2> part(static_cast<size_t>(B) * m1 * nblk);
    DevBuf<double> part2(static_cast<size_t>(B) * nblk), est(B), inv(B), nrm(B);
    DevBuf<int32_t> cols_d(B), jn_d(B);
    LSPR_HIP(hipMemsetAsync(x, 0, B * nvec * sizeof(double2), s));

    SolveResult res;
    res.iters.assign(B, 0);
    res.rel_resid.assign(B, 0.0);
    std::vector<int32_t> jn(B, 0);
    std::vector<double> bnorm(B), est_h(B), nrm_h(B);

    auto upload_cols = [&](const std::vector<int32_t>& c) {
        LSPR_HIP(hipMemcpyAsync(cols_d.p, c.data(), c.size() * 4, hipMemcpyHostToDevice, s));
    };
    auto norms = [&](const double2* vec, int64_t stride, const std::vector<int32_t>& c) {
        upload_cols(c);
        const int ns = static_cast<int>(c.size());
        hipLaunchKernelGGL(k_norm_part, dim3(nblk, ns), dim3(GT), 0, s, vec, nvec, stride,
                           cols_d.p, part2.p, nblk);
        hipLaunchKernelGGL(k_norm_final, dim3((ns + 63) / 64), dim3(64), 0, s, part2.p, nblk,
                           cols_d.p, ns, nrm.p, inv.p);
        LSPR_HIP(hipGetLastError());
        LSPR_HIP(hipMemcpyAsync(nrm_h.data(), nrm.p, B * 8, hipMemcpyDeviceToHost, s));
        LSPR_HIP(hipStreamSynchronize(s));
    };

    // b, ||b||; r0 = b goes to V_0 after scaling
    if (b_in != nullptr)
        LSPR_HIP(hipMemcpyAsync(bvec.p, b_in, B * nvec * sizeof(double2), hipMemcpyDeviceToDevice, s));
    else
        system_rhs(g, B, ratio_d, e_field, bvec.p, nvec, s);
    std::vector<int32_t> active(B);
    for (int b = 0; b < B; ++b) active[b] = b;
    norms(bvec.p, nvec, active);
    bnorm = nrm_h;
    {
        std::vector<int32_t> keep;
        for (int b : active)
            if (bnorm[b] > 0.0) keep.push_back(b);
        active.swap(keep);
    }
    if (!active.empty()) {
        upload_cols(active);
        const int ns = static_cast<int>(active.size());
        hipLaunchKernelGGL(k_scale, dim3(nblk, ns), dim3(GT), 0, s, bvec.p, nvec, V.p,
                           m1 * nvec, nvec, cols_d.p, inv.p);
        hipLaunchKernelGGL(k_set_g, dim3((ns * m1 + 255) / 256), dim3(256), 0, s, gv.p, m1,
                           cols_d.p, ns, nrm.p);
        LSPR_HIP(hipGetLastError());
    }
    while (!active.empty()) {
        // ---------------- one restart cycle over the active columns
        std::vector<int32_t> running = active;
        for (int b : active) jn[b] = 0;
        for (int j = 0; j < m && !running.empty(); ++j) {
            upload_cols(running);
            const int ns = static_cast<int>(running.size());
            const double2* vin = V.p + j * nvec;
            int64_t vin_stride = m1 * nvec;
            if (pre) {
                const int64_t t = static_cast<int64_t>(g.N) * ns;
                hipLaunchKernelGGL(k_precond, dim3((t + 255) / 256), dim3(256), 0, s, vin,
                                   vin_stride, z.p, nvec, g.N, cols_d.p, ns, ratio_d, g.S,
                                   g.surf.p, g.vself.p, 0);
                LSPR_HIP(hipGetLastError());
                vin = z.p;
                vin_stride = nvec;
            }
            system_apply(g, prec, ns, ratio_d, vin, vin_stride, w.p, nvec, cols_d.p, s);
            {
                // two sweeps reading j+1 basis vectors twice each (dots, update) plus w
                prof::Scope sc("arnoldi", s, 2.0 * 16.0 * (j + 1) * double(nvec) * ns,
                               (4.0 * (j + 1) + 8.0) * 16.0 * double(nvec) * ns);
                for (int pass = 0; pass < 2; ++pass) {
                    hipLaunchKernelGGL(k_dots, dim3(nblk, ns), dim3(GT),
                                       (GT / 64) * (j + 1) * sizeof(double2), s, V.p, m1, nvec, j,
                                       w.p, cols_d.p, part.p, nblk);
                    const int nt = ns * (j + 1);
                    hipLaunchKernelGGL(k_dots_final, dim3((nt + 255) / 256), dim3(256), 0, s, part.p,
                                       nblk, m1, j, cols_d.p, ns, hpass.p, hcol.p, pass);
                    hipLaunchKernelGGL(k_update, dim3(nblk, ns), dim3(GT), 0, s, V.p, m1, nvec, j,
                                       w.p, cols_d.p, hpass.p);
                    LSPR_HIP(hipGetLastError());
            }
            hipLaunchKernelGGL(k_norm_part, dim3(nblk, ns), dim3(GT), 0, s, w.p, nvec, nvec,
                               cols_d.p, part2.p, nblk);
            hipLaunchKernelGGL(k_arnoldi_finish, dim3((ns + 63) / 64), dim3(64), 0, s, part2.p,
                               nblk, cols_d.p, ns, m, j, hcol.p, H.p, cs.p, sn.p, gv.p, est.p,
                               inv.p);
            hipLaunchKernelGGL(k_scale, dim3(nblk, ns), dim3(GT), 0, s, w.p, nvec,
                               V.p + (j + 1) * nvec, m1 * nvec, nvec, cols_d.p, inv.p);
            LSPR_HIP(hipGetLastError());
            }
            LSPR_HIP(hipMemcpyAsync(est_h.data(), est.p, B * 8, hipMemcpyDeviceToHost, s));
            LSPR_HIP(hipStreamSynchronize(s));
            std::vector<int32_t> still;
            for (int b : running) {
                jn[b] = j + 1;
                res.iters[b] += 1;
                const bool done = est_h[b] <= gm.tol * bnorm[b] || res.iters[b] >= gm.max_iter;
                if (!done) still.push_back(b);
            }
            running.swap(still);
        }
        // ---------------- solution update x += M^{-1} V y and true residual
        upload_cols(active);
        const int ns = static_cast<int>(active.size());
        LSPR_HIP(hipMemcpyAsync(jn_d.p, jn.data(), B * 4, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_backsolve, dim3((ns + 63) / 64), dim3(64), 0, s, H.p, gv.p, jn_d.p,
                           cols_d.p, ns, m, y.p);
        hipLaunchKernelGGL(k_basis_combine, dim3(nblk, ns), dim3(GT), 0, s, V.p, m1, nvec, y.p,
                           m, jn_d.p, cols_d.p, w.p);
        LSPR_HIP(hipGetLastError());
        if (pre) {
            const int64_t t = static_cast<int64_t>(g.N) * ns;
            hipLaunchKernelGGL(k_precond, dim3((t + 255) / 256), dim3(256), 0, s, w.p, nvec, x,
                               nvec, g.N, cols_d.p, ns, ratio_d, g.S, g.surf.p, g.vself.p, 1);
        } else {
            hipLaunchKernelGGL(k_axpy, dim3(nblk, ns), dim3(GT), 0, s, w.p, x, nvec, cols_d.p);
        }
        LSPR_HIP(hipGetLastError());
        system_apply(g, prec, ns, ratio_d, x, nvec, w.p, nvec, cols_d.p, s);
        hipLaunchKernelGGL(k_resid, dim3(nblk, ns), dim3(GT), 0, s, bvec.p, w.p, V.p, m1 * nvec,
                           nvec, cols_d.p);
        LSPR_HIP(hipGetLastError());
        norms(V.p, m1 * nvec, active);
        std::vector<int32_t> cont;
        for (int b : active) {
            res.rel_resid[b] = nrm_h[b] / bnorm[b];
            if (res.rel_resid[b] <= gm.tol) continue;
            if (res.iters[b] >= gm.max_iter) {
                res.all_converged = false;
                continue;
            }
            cont.push_back(b);
        }
        active.swap(cont);
        if (!active.empty()) {
            upload_cols(active);
            const int ns2 = static_cast<int>(active.size());
            hipLaunchKernelGGL(k_scale, dim3(nblk, ns2), dim3(GT), 0, s, V.p, m1 * nvec, V.p,
                               m1 * nvec, nvec, cols_d.p, inv.p);
            hipLaunchKernelGGL(k_set_g, dim3((ns2 * m1 + 255) / 256), dim3(256), 0, s, gv.p, m1,
                               cols_d.p, ns2, nrm.p);
            LSPR_HIP(hipGetLastError());
        }
    }
    LSPR_HIP(hipStreamSynchronize(s));
    return res;
}

// Mixed-precision iterative refinement: x_{k+1} = x_k + d_k, where d_k solves A d = r_k by
// GMRES with FP32 far-field products to the relative tolerance inner_tol, and the residual
// r_k = b - A x_k is formed with FP64 products.  A column stops when ||r_k|| <= tol ||b|| or its
// total inner iterations reach max_iter.
SolveResult refine_solve(Geometry& g, int B, const double2* ratio_d, const double* e_field,
                         const lspr_gmres_params& gm, double2* x, hipStream_t s) {
    const int64_t nvec = 2 * static_cast<int64_t>(g.N);
    const int nblk = blocks_for(nvec);
    DevBuf<double2> b(B * nvec), r(B * nvec), d(B * nvec), w(B * nvec);
    DevBuf<double> part2(static_cast<size_t>(B) * nblk), nrm(B), inv(B);
    DevBuf<int32_t> cols_d(B);
    std::vector<double> nrm_h(B);
    LSPR_HIP(hipMemsetAsync(x, 0, B * nvec * sizeof(double2), s));
    auto norms = [&](const double2* vec, const std::vector<int32_t>& c) {
        LSPR_HIP(hipMemcpyAsync(cols_d.p, c.data(), c.size() * 4, hipMemcpyHostToDevice, s));
        const int ns = static_cast<int>(c.size());
        hipLaunchKernelGGL(k_norm_part, dim3(nblk, ns), dim3(GT), 0, s, vec, nvec, nvec,
                           cols_d.p, part2.p, nblk);
        hipLaunchKernelGGL(k_norm_final, dim3((ns + 63) / 64), dim3(64), 0, s, part2.p, nblk,
                           cols_d.p, ns, nrm.p, inv.p);
        LSPR_HIP(hipGetLastError());
        LSPR_HIP(hipMemcpyAsync(nrm_h.data(), nrm.p, B * 8, hipMemcpyDeviceToHost, s));
        LSPR_HIP(hipStreamSynchronize(s));
    };
    system_rhs(g, B, ratio_d, e_field, b.p, nvec, s);
    LSPR_HIP(hipMemcpyAsync(r.p, b.p, B * nvec * sizeof(double2), hipMemcpyDeviceToDevice, s));
    std::vector<int32_t> active(B);
    for (int c = 0; c < B; ++c) active[c] = c;
    norms(b.p, active);
    const std::vector<double> bnorm = nrm_h;
    SolveResult res;
    res.iters.assign(B, 0);
    res.rel_resid.assign(B, 0.0);
    auto retire = [&](int c) {  // a zero residual column is skipped by the inner solves
        LSPR_HIP(hipMemsetAsync(r.p + c * nvec, 0, nvec * sizeof(double2), s));
    };
    {
        std::vector<int32_t> keep;
        for (int c : active) {
            if (bnorm[c] > 0.0) keep.push_back(c);
            else retire(c);
        }
        active.swap(keep);
    }
    lspr_gmres_params gi = gm;
    gi.tol = gm.inner_tol > 0.0 ? gm.inner_tol : 1e-4;
    for (int outer = 0; !active.empty(); ++outer) {
        int used = 0;
        for (int c : active) used = std::max(used, res.iters[c]);
        gi.max_iter = std::max(1, gm.max_iter - used);
        const SolveResult ri = gmres_solve(g, LSPR_FP32, B, ratio_d, e_field, gi, r.p, d.p, s);
        for (int c : active) res.iters[c] += ri.iters[c];
        LSPR_HIP(hipMemcpyAsync(cols_d.p, active.data(), active.size() * 4,
                                hipMemcpyHostToDevice, s));
        const int ns = static_cast<int>(active.size());
        hipLaunchKernelGGL(k_axpy, dim3(nblk, ns), dim3(GT), 0, s, d.p, x, nvec, cols_d.p);
        LSPR_HIP(hipGetLastError());
        system_apply(g, LSPR_FP64, ns, ratio_d, x, nvec, w.p, nvec, cols_d.p, s);
        hipLaunchKernelGGL(k_resid, dim3(nblk, ns), dim3(GT), 0, s, b.p, w.p, r.p, nvec, nvec,
                           cols_d.p);
        LSPR_HIP(hipGetLastError());
        norms(r.p, active);
        std::vector<int32_t> cont;
        for (int c : active) {
            res.rel_resid[c] = nrm_h[c] / bnorm[c];
            if (res.rel_resid[c] <= gm.tol) {
                retire(c);
                continue;
            }
            if (res.iters[c] >= gm.max_iter || outer >= 50) {
                res.all_converged = false;
                retire(c);
                continue;
            }
            cont.push_back(c);
        }
        active.swap(cont);
    }
    LSPR_HIP(hipStreamSynchronize(s));
    return res;
}

}  // namespace lspr
