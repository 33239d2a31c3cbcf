// Batched restarted GMRES in complex FP64 (section "Code modifications and added features":
// the solver accepts complex numbers; the paper fixes only tolerances, Tables 2 and 5).
//
// Every wavelength has its own Krylov space; all running wavelengths share each block
// matrix-vector product.  The Arnoldi process runs on the device as classical Gram-Schmidt with
// delayed re-orthogonalisation (the low-synchronisation "DCGS2" scheme of Swirydowicz et al.,
// 2020, and Bielich et al., 2022), written out below from its defining relations.  Step j
// multiplies the provisional vector p (slot j: projected once against q_0..q_{j-1} and
// normalised) and then needs one pass over the basis for all inner products
//     s = Q^H p,  alpha = p^H p,  z = Q^H w,  beta = p^H w,  gamma = w^H w   (w = A p)
// and one pass that writes the final q_j = (p - Q s) / r, r = sqrt(alpha - |s|^2), and the next
// provisional vector.  With p = Q s + r q_j the relations
//     A q_j = (w - Q_{0..j} H s) / r,      u_j = (w - Q (z - s t) - p t) / r,
//     t = (beta - s^H z) / r^2,             |u_j|^2 = (gamma - |z|^2 - r^2 |t|^2) / r^2
// give Hessenberg column j (provisional until its subdiagonal norm is corrected one step
// later: column j-1 becomes final as h_{:,j-1} += |u_{j-1}| s, h_{j,j-1} = |u_{j-1}| r).  So each
// step reads the basis twice instead of four times (classical Gram-Schmidt with a second pass),
// with the same orthogonality.  Givens rotations turn each final column; the residual estimate
// of the next dimension is predicted from the provisional column, and when it meets the
// tolerance (or the cycle or the iteration budget ends) the column is finalised with an inner
// product pass alone, so no matrix-vector product is wasted.  The host only launches kernels
// and reads two residual estimates per wavelength per step to retire converged wavelengths,
// which then leave the matrix-vector product.  With LSPR_FP32_LEAD64 a wavelength's product
// runs in FP64 while its residual estimate is above a level (inner_tol, default 0.3, relative
// to ||b||) and in FP32 after: the error of the product of basis vector q_j reaches the
// solution scaled by its coefficient y_j, and these fall with the residual (the relaxation
// results for inexact Krylov methods: Simoncini and Szyld 2003, van den Eshof and Sleijpen
// 2004), so only the first few products need FP64.  x0 = 0; a wavelength stops when
// ||b - A x|| <= tol ||b||, checked on the true residual at each restart.  Optional right
// block-Jacobi preconditioning with the 2x2 self-panel blocks (K_ii = 0 on flat panels) does not
// change the solution.
#include <algorithm>
#include <cmath>

#include "precond.hpp"
#include "profile.hpp"
#include "system.hpp"

namespace lspr {

namespace {

constexpr int GT = 256;
constexpr int FT = 256, FR = 8;  // finishing kernel: threads, threads per partial-sum reduction
constexpr int GE = 16;
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

// Inner products of one Arnoldi step.  nq final basis vectors Q = V_0..V_{nq-1}, the provisional
// vector p = V_nq and (WITH_W) the product w.  Per wave and block slice, partial sums of
//   k < nq: q_k^H p;  k = nq: p^H p;  (WITH_W) nq + 1 + k: q_k^H w;  2 nq + 1: p^H w;  2 nq + 2: w^H w
// go to part[(slot * kmax + k) * nparts + 4 blk + wave].  The basis is taken KB vectors at a
// time, and the wave reductions of their 4 KB partial sums are interleaved, so that the
// cross-lane exchanges overlap instead of waiting on each other.
template <int WITH_W>
__global__ void __launch_bounds__(GT) k_dcgs_red(const double2* __restrict__ V, int m1,
                                                 int64_t nvec, int nq,
                                                 const double2* __restrict__ w,
                                                 const int32_t* __restrict__ cols,
                                                 double2* __restrict__ part, int kmax,
                                                 int nparts) {
    constexpr int KB = 4, NV = WITH_W ? 4 : 2;  // values per basis vector: s (re, im) [, z]
    const int slot = blockIdx.y, col = cols[slot];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * GSLICE;
    const double2* Vc = V + static_cast<int64_t>(col) * m1 * nvec;
    const double2* wc = w + col * nvec;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double2* out = part + static_cast<int64_t>(slot) * kmax * nparts + 4 * blockIdx.x + wave;
    // element indices clamped into the vector and out-of-range values zeroed by a select, so
    // that loads carry no branch and all of a step's loads are in flight together
    int64_t nn[GE];
    bool in[GE];
    double2 pl[GE], wl[GE];
#pragma unroll
    for (int e = 0; e < GE; ++e) {
        const int64_t n = base + e * GT + threadIdx.x;
        in[e] = n < nvec;
        nn[e] = in[e] ? n : nvec - 1;
    }
#pragma unroll
    for (int e = 0; e < GE; ++e) {
        const double2 a = Vc[nq * nvec + nn[e]];
        pl[e] = in[e] ? a : make_double2(0.0, 0.0);
        if constexpr (WITH_W) {
            const double2 c = wc[nn[e]];
            wl[e] = in[e] ? c : make_double2(0.0, 0.0);
        } else {
            wl[e] = make_double2(0.0, 0.0);
        }
    }
    for (int k0 = 0; k0 < nq; k0 += KB) {
        double v[KB][NV];
#pragma unroll
        for (int kk = 0; kk < KB; ++kk) {
#pragma unroll
            for (int c = 0; c < NV; ++c) v[kk][c] = 0.0;
            // past the last basis vector the products read vector nq - 1 again and are dropped
            const int k = k0 + kk < nq ? k0 + kk : nq - 1;
            const double2* qk = Vc + k * nvec;
            double2 q[GE];
#pragma unroll
            for (int e = 0; e < GE; ++e) q[e] = qk[nn[e]];  // pl, wl are zero out of range
#pragma unroll
            for (int e = 0; e < GE; ++e) {
                const double2 a = cconjmul(q[e], pl[e]);
                v[kk][0] += a.x;
                v[kk][1] += a.y;
                if constexpr (WITH_W) {
                    const double2 c = cconjmul(q[e], wl[e]);
                    v[kk][2] += c.x;
                    v[kk][3] += c.y;
                }
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int kk = 0; kk < KB; ++kk)
#pragma unroll
                for (int c = 0; c < NV; ++c) v[kk][c] += __shfl_xor(v[kk][c], off, 64);
        if (lane == 0) {
#pragma unroll
            for (int kk = 0; kk < KB; ++kk) {
                const int k = k0 + kk;
                if (k < nq) {
                    out[static_cast<int64_t>(k) * nparts] = make_double2(v[kk][0], v[kk][1]);
                    if constexpr (WITH_W)
                        out[static_cast<int64_t>(nq + 1 + k) * nparts] = make_double2(v[kk][2], v[kk][3]);
                }
            }
        }
    }
    double al = 0.0, br = 0.0, bi = 0.0, ga = 0.0;
#pragma unroll
    for (int e = 0; e < GE; ++e) {
        al += pl[e].x * pl[e].x + pl[e].y * pl[e].y;
        const double2 c = cconjmul(pl[e], wl[e]);
        br += c.x;
        bi += c.y;
        ga += wl[e].x * wl[e].x + wl[e].y * wl[e].y;
    }
    al = wave_sum(al);
    if constexpr (WITH_W) {
        br = wave_sum(br);
        bi = wave_sum(bi);
        ga = wave_sum(ga);
    }
    if (lane == 0) {
        out[static_cast<int64_t>(nq) * nparts] = make_double2(al, 0.0);
        if constexpr (WITH_W) {
            out[static_cast<int64_t>(2 * nq + 1) * nparts] = make_double2(br, bi);
            out[static_cast<int64_t>(2 * nq + 2) * nparts] = make_double2(ga, 0.0);
        }
    }
}

// Per-wavelength state of the Arnoldi process (all arrays indexed by column col):
//   Hr [m][m1]  final Hessenberg columns as the Arnoldi relation has them (not rotated)
//   H  [m][m1]  the same columns after the Givens rotations (upper triangle for the back solve)
//   hp [m1 + 1] the provisional column, nu its provisional subdiagonal |u|
//   cs, sn [m]  rotations; gv [m1] rotated right-hand side |r0| e_0
//   coef [kmax] update coefficients: s (m1), z - s t (m1), then 1/r, t, 1/(r nu)
struct ArnoldiState {
    double2 *Hr, *H, *hp, *cs, *sn, *gv, *coef;
    double *nu, *est_fin, *est_prov, *r_fin;
    int32_t* fin;
    int m, kmax;
};

// Applies the rotations 0..c-1 (cs, sn) to column h (entries 0..c+1) and returns the rotation
// that zeroes h[c + 1] (h[c] becomes its norm).
__device__ void rotate_column(double2* h, int c, const double2* cs, const double2* sn,
                              double2& cc, double2& ss) {
    for (int i = 0; i < c; ++i) {  // [x, y] -> [conj(c) x + conj(s) y, -s x + c y]
        const double2 hi = h[i], hn = h[i + 1];
        const double2 a = cconjmul(cs[i], hi), bq = cconjmul(sn[i], hn);
        const double2 d = cmul(sn[i], hi), e = cmul(cs[i], hn);
        h[i] = make_double2(a.x + bq.x, a.y + bq.y);
        h[i + 1] = make_double2(e.x - d.x, e.y - d.y);
    }
    const double2 a = h[c], bq = h[c + 1];
    const double den = sqrt(a.x * a.x + a.y * a.y + bq.x * bq.x + bq.y * bq.y);
    cc = make_double2(1.0, 0.0);
    ss = make_double2(0.0, 0.0);
    if (den > 0.0) {
        cc = make_double2(a.x / den, a.y / den);
        ss = make_double2(bq.x / den, bq.y / den);
    }
    h[c] = make_double2(den, 0.0);
    h[c + 1] = make_double2(0.0, 0.0);
}

// One block of 64 threads per running column; it first adds the inner products' partial sums
// (in a fixed order) and stages the column's rotations and provisional Hessenberg column in LDS,
// so that the sequential part (thread 0) touches LDS only.
// mode 0, step j (nq = j): finalise column j - 1 (unless a finalising pass already did), form
//   provisional column j, the update coefficients and the predicted estimate of dimension j + 1.
// mode 1, step j (nq = j + 1): finalise column j only.
// Finalising column c: h_{i,c} = hp_i + nu s_i (i <= c), h_{c+1,c} = nu r; stored raw and
// rotated, with the rotated right-hand side and the final residual estimate.
__global__ void __launch_bounds__(FT) k_dcgs_finish(const double2* __restrict__ part, int nparts,
                                                    const int32_t* __restrict__ cols, int mode,
                                                    int j, ArnoldiState A) {
    extern __shared__ double2 sh[];  // rd [kmax], g [m1 + 1], tmp [m1 + 1], cs [m], sn [m], hp [m1 + 1]
    const int slot = blockIdx.x, col = cols[slot];
    const int m = A.m, m1 = m + 1, tid = threadIdx.x;
    double2* rd = sh;
    double2* g = rd + A.kmax;
    double2* tmp = g + m1 + 1;
    double2* csl = tmp + m1 + 1;
    double2* snl = csl + m;
    double2* hpl = snl + m;
    const int nq = mode == 0 ? j : j + 1;
    const int nk = mode == 0 ? 2 * nq + 3 : nq + 1;
    const int c = mode == 0 ? j - 1 : j;  // the column to finalise (none when c < 0)
    __shared__ double r_sh;
    __shared__ int fin_sh;
    // partial sums: FR consecutive threads per sum, each adding every FR-th partial, then
    // combined across the FR threads in a fixed order (so that the loads are in flight together)
    for (int k0 = 0; k0 < nk; k0 += FT / FR) {
        const int k = k0 + tid / FR, sub = tid % FR;
        double2 acc = make_double2(0.0, 0.0);
        if (k < nk) {
            const double2* p = part + (static_cast<int64_t>(slot) * A.kmax + k) * nparts;
#pragma unroll 8
            for (int b = sub; b < nparts; b += FR) {
                acc.x += p[b].x;
                acc.y += p[b].y;
            }
        }
#pragma unroll
        for (int off = FR / 2; off > 0; off >>= 1) {
            acc.x += __shfl_xor(acc.x, off, 64);
            acc.y += __shfl_xor(acc.y, off, 64);
        }
        if (k < nk && sub == 0) rd[k] = acc;
    }
    const int nrot = mode == 0 ? j : j + 1;  // rotations a step may read (0..c, then c)
    for (int i = tid; i < nrot && i < m; i += FT) {
        csl[i] = A.cs[col * m + i];
        snl[i] = A.sn[col * m + i];
    }
    for (int i = tid; i <= j + 1 && i <= m1; i += FT) hpl[i] = A.hp[static_cast<int64_t>(col) * (m1 + 1) + i];
    __syncthreads();
    const double2* s = rd;                // s_i = q_i^H p, i < nq
    const double2* z = rd + nq + 1;       // z_i = q_i^H w, i < nq (mode 0)
    if (tid == 0) {
        double ss = 0.0;
        for (int i = 0; i < nq; ++i) ss += s[i].x * s[i].x + s[i].y * s[i].y;
        const double r = sqrt(fmax(rd[nq].x - ss, 0.0));
        r_sh = r;
        const bool do_fin = c >= 0 && (mode == 1 || A.fin[col] != c);
        fin_sh = do_fin;
        if (do_fin) {
            const double nu = A.nu[col];
            for (int i = 0; i <= c; ++i)
                tmp[i] = make_double2(hpl[i].x + nu * s[i].x, hpl[i].y + nu * s[i].y);
            tmp[c + 1] = make_double2(nu * r, 0.0);
            for (int i = 0; i <= c + 1; ++i) g[i] = tmp[i];  // raw copy (g is free until later)
            double2 cc, sr;
            rotate_column(tmp, c, csl, snl, cc, sr);
            csl[c] = cc;
            snl[c] = sr;
            A.cs[col * m + c] = cc;
            A.sn[col * m + c] = sr;
            double2* gv = A.gv + col * m1;
            const double2 gc = gv[c];
            const double2 t = cmul(sr, gc);
            gv[c + 1] = make_double2(-t.x, -t.y);
            gv[c] = cconjmul(cc, gc);
            A.est_fin[col] = sqrt(t.x * t.x + t.y * t.y);
            A.fin[col] = c;
            A.r_fin[col] = r;
            if (mode == 1) A.est_prov[col] = A.est_fin[col];
        }
    }
    __syncthreads();
    if (fin_sh) {  // column c, raw (in g) and rotated (in tmp)
        double2* hr = A.Hr + (static_cast<int64_t>(col) * m + c) * m1;
        double2* H = A.H + (static_cast<int64_t>(col) * m + c) * m1;
        for (int i = tid; i <= c + 1; i += FT) {
            hr[i] = g[i];
            H[i] = tmp[i];
        }
    }
    if (mode == 1) return;
    __syncthreads();  // column j - 1 of Hr is in memory before g reads it
    const double r = r_sh;
    // g = Hr[0..j][0..j-1] s (column k of Hr has entries 0..k+1)
    const double2* hr = A.Hr + static_cast<int64_t>(col) * m * m1;
    for (int i = tid; i <= j; i += FT) {
        double2 acc = make_double2(0.0, 0.0);
        for (int k = (i > 0 ? i - 1 : 0); k < j; ++k) {
            const double2 p = cmul(hr[k * m1 + i], s[k]);
            acc.x += p.x;
            acc.y += p.y;
        }
        g[i] = acc;
    }
    __syncthreads();
    double2* coef = A.coef + col * A.kmax;
    __shared__ double2 t_sh;
    if (tid == 0) {
        if (!(r > 0.0)) {  // p lies in the span of Q: the space is invariant (breakdown)
            t_sh = make_double2(0.0, 0.0);
            coef[2 * m1] = coef[2 * m1 + 1] = coef[2 * m1 + 2] = make_double2(0.0, 0.0);
            A.est_prov[col] = 0.0;
        } else {
            const double beta_r = rd[2 * nq + 1].x, beta_i = rd[2 * nq + 1].y, gamma = rd[2 * nq + 2].x;
            double2 sz = make_double2(0.0, 0.0);
            double zz = 0.0;
            for (int i = 0; i < j; ++i) {
                const double2 q = cconjmul(s[i], z[i]);
                sz.x += q.x;
                sz.y += q.y;
                zz += z[i].x * z[i].x + z[i].y * z[i].y;
            }
            const double inv_r = 1.0 / r;
            const double2 qw = make_double2((beta_r - sz.x) * inv_r, (beta_i - sz.y) * inv_r);  // q_j^H w
            const double2 t = make_double2(qw.x * inv_r, qw.y * inv_r);
            t_sh = t;
            for (int i = 0; i < j; ++i)
                hpl[i] = make_double2((z[i].x - g[i].x) * inv_r, (z[i].y - g[i].y) * inv_r);
            hpl[j] = make_double2((qw.x - g[j].x) * inv_r, (qw.y - g[j].y) * inv_r);
            const double nu2 = gamma - zz - (qw.x * qw.x + qw.y * qw.y);
            const double nu = sqrt(fmax(nu2, 1e-30 * gamma)) * inv_r;
            hpl[j + 1] = make_double2(nu, 0.0);
            A.nu[col] = nu;
            coef[2 * m1] = make_double2(inv_r, 0.0);
            coef[2 * m1 + 1] = t;
            coef[2 * m1 + 2] = make_double2(nu > 0.0 ? inv_r / nu : 0.0, 0.0);
            // predicted estimate of dimension j + 1 from the provisional column
            for (int i = 0; i <= j + 1; ++i) tmp[i] = hpl[i];
            double2 cc, ssr;
            rotate_column(tmp, j, csl, snl, cc, ssr);
            const double2 gj = A.gv[col * m1 + j];
            A.est_prov[col] = sqrt(ssr.x * ssr.x + ssr.y * ssr.y) * sqrt(gj.x * gj.x + gj.y * gj.y);
        }
    }
    __syncthreads();
    const bool ok = r > 0.0;
    const double2 t = t_sh;
    double2* hp = A.hp + static_cast<int64_t>(col) * (m1 + 1);
    for (int i = tid; i < j; i += FT) {
        const double2 st = cmul(s[i], t);
        coef[i] = ok ? s[i] : make_double2(0.0, 0.0);
        coef[m1 + i] = ok ? make_double2(z[i].x - st.x, z[i].y - st.y) : make_double2(0.0, 0.0);
    }
    if (ok)
        for (int i = tid; i <= j + 1; i += FT) hp[i] = hpl[i];
}

// Second pass of step j: q_j = (p - Q s) / r into slot j and the next provisional vector
// (w - Q (z - s t) - p t) / (r nu) into slot j + 1, reading each basis vector once.
__global__ void __launch_bounds__(GT) k_dcgs_update(double2* __restrict__ V, int m1, int64_t nvec,
                                                    int j, const double2* __restrict__ w,
                                                    const int32_t* __restrict__ cols,
                                                    const double2* __restrict__ coef, int kmax) {
    extern __shared__ double2 cfs[];  // [2 j]: s, then z - s t
    const int col = cols[blockIdx.y];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * GSLICE;
    double2* Vc = V + static_cast<int64_t>(col) * m1 * nvec;
    const double2* cf = coef + col * kmax;
    for (int i = threadIdx.x; i < j; i += GT) {
        cfs[i] = cf[i];
        cfs[j + i] = cf[m1 + i];
    }
    __syncthreads();
    const double qs = cf[2 * m1].x, ws = cf[2 * m1 + 2].x;
    const double2 t = cf[2 * m1 + 1];
    // basis vector by basis vector, GE elements per thread, so that GE loads are in flight
    // clamped indices: loads without branches (out-of-range lanes compute values never stored)
    int64_t nn[GE];
#pragma unroll
    for (int e = 0; e < GE; ++e) {
        const int64_t n = base + e * GT + threadIdx.x;
        nn[e] = n < nvec ? n : nvec - 1;
    }
    double2 aq[GE], aw[GE];
#pragma unroll
    for (int e = 0; e < GE; ++e) {
        const double2 p = Vc[j * nvec + nn[e]];
        const double2 wv = w[col * nvec + nn[e]];
        const double2 pt = cmul(t, p);
        aq[e] = p;
        aw[e] = make_double2(wv.x - pt.x, wv.y - pt.y);
    }
#pragma unroll 2
    for (int i = 0; i < j; ++i) {
        const double2* qi = Vc + i * nvec;
        const double2 cq = cfs[i], cw = cfs[j + i];
        double2 qv[GE];
#pragma unroll
        for (int e = 0; e < GE; ++e) qv[e] = qi[nn[e]];
#pragma unroll
        for (int e = 0; e < GE; ++e) {
            const double2 q = qv[e];
            const double2 a = cmul(cq, q), c = cmul(cw, q);
            aq[e].x -= a.x;
            aq[e].y -= a.y;
            aw[e].x -= c.x;
            aw[e].y -= c.y;
        }
    }
#pragma unroll
    for (int e = 0; e < GE; ++e) {
        const int64_t n = base + e * GT + threadIdx.x;
        if (n < nvec) {
            Vc[j * nvec + n] = make_double2(aq[e].x * qs, aq[e].y * qs);
            Vc[(j + 1) * nvec + n] = make_double2(aw[e].x * ws, aw[e].y * ws);
        }
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
// One 64-thread block per column: column-oriented back substitution, the right-hand side in
// LDS (y_k from the finished r_k, then r_i -= H_ik y_k for all i < k in parallel).
__global__ void __launch_bounds__(64) k_backsolve(const double2* __restrict__ H,
                                                  const double2* __restrict__ gv,
                                                  const int32_t* __restrict__ jn,
                                                  const int32_t* __restrict__ cols, int m,
                                                  double2* __restrict__ y) {
    extern __shared__ double2 rs[];  // [m + 1]
    const int col = cols[blockIdx.x], tid = threadIdx.x;
    const int n = jn[col], m1 = m + 1;
    const double2* Hc = H + static_cast<int64_t>(col) * m * m1;  // column k at Hc + k*m1
    double2* yc = y + col * m;
    for (int i = tid; i < n; i += 64) rs[i] = gv[col * m1 + i];
    __syncthreads();
    for (int k = n - 1; k >= 0; --k) {
        const double2 d = Hc[k * m1 + k];
        const double2 yk = (d.x == 0.0 && d.y == 0.0) ? make_double2(0.0, 0.0) : cdiv(rs[k], d);
        if (tid == 0) yc[k] = yk;
        for (int i = tid; i < k; i += 64) {
            const double2 p = cmul(Hc[k * m1 + i], yk);
            rs[i].x -= p.x;
            rs[i].y -= p.y;
        }
        __syncthreads();
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
    double2 phi, psi;
    block_jacobi(a, b, ratio[col * S + surf[i]], vself[i] * INV_4PI, phi, psi);
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

// Pinned host memory for the residual estimates, one block per host thread, allocated once and
// kept for the life of the process (freeing pinned memory can wait for the whole device, which
// would stall concurrent requests).
double* pinned_estimates(int n) {
    constexpr int CAP = 4 * 64;
    LSPR_REQUIRE(n <= CAP, LSPR_E_INVALID, "too many columns for the estimate buffer");
    thread_local double* p = nullptr;
    if (p == nullptr)
        LSPR_HIP(hipHostMalloc(reinterpret_cast<void**>(&p), CAP * sizeof(double), hipHostMallocDefault));
    return p;
}

// Column lists go to the device through a ring of pinned slots (asynchronous copies); a slot is
// reused only after the event recorded behind its last copy has completed.  Per host thread,
// allocated once and kept.
struct PinnedCols {
    static constexpr int SLOTS = 8, CAP = 64;
    int32_t* host = nullptr;
    hipEvent_t ev[SLOTS] = {};
    int next = 0, dev = -1;
    void upload(int32_t* dst, const std::vector<int32_t>& c, hipStream_t s) {
        LSPR_REQUIRE(static_cast<int>(c.size()) <= CAP, LSPR_E_INVALID, "too many columns");
        int d = 0;
        LSPR_HIP(hipGetDevice(&d));
        if (host != nullptr && d != dev) {  // events belong to one device: plain copy elsewhere
            LSPR_HIP(hipMemcpyAsync(dst, c.data(), c.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, s));
            return;
        }
        if (host == nullptr) {
            dev = d;
            LSPR_HIP(hipHostMalloc(reinterpret_cast<void**>(&host), SLOTS * CAP * sizeof(int32_t),
                                   hipHostMallocDefault));
            for (hipEvent_t& e : ev) LSPR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        }
        const int k = next;
        next = (next + 1) % SLOTS;
        LSPR_HIP(hipEventSynchronize(ev[k]));
        std::copy(c.begin(), c.end(), host + k * CAP);
        LSPR_HIP(hipMemcpyAsync(dst, host + k * CAP, c.size() * sizeof(int32_t),
                                hipMemcpyHostToDevice, s));
        LSPR_HIP(hipEventRecord(ev[k], s));
    }
};
PinnedCols& pinned_cols() {
    thread_local PinnedCols pc;
    return pc;
}

struct Event {
    hipEvent_t e = nullptr;
    Event() { LSPR_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming)); }
    ~Event() { (void)hipEventDestroy(e); }
    Event(const Event&) = delete;
    Event& operator=(const Event&) = delete;
};

}  // namespace

SolveResult gmres_solve(Geometry& g, int prec, int B, const double2* ratio_d,
                        const double* e_field, const lspr_gmres_params& gm, const double2* b_in,
                        double2* x, hipStream_t s) {
    const int m = gm.restart, m1 = m + 1;
    const int64_t nvec = 2 * static_cast<int64_t>(g.N);
    const int nblk = blocks_for(nvec);
    const bool pre = gm.precond != 0;
    DevBuf<double2> V(static_cast<size_t>(B) * m1 * nvec), w(B * nvec), bvec(B * nvec);
    const int kmax = 2 * m1 + 3;
    const int nparts = 4 * nblk;  // one partial sum per wave of each block
    DevBuf<double2> Hr(static_cast<size_t>(B) * m * m1), H(static_cast<size_t>(B) * m * m1);
    DevBuf<double2> hp(B * (m1 + 1)), cs(B * m), sn(B * m), gv(B * m1), y(B * m);
    DevBuf<double2> coef(B * kmax);
    DevBuf<double2> part(static_cast<size_t>(B) * kmax * nparts);
    DevBuf<double> part2(static_cast<size_t>(B) * nblk), inv(B), nrm(B);
    DevBuf<double> nu(B), est(2 * B), r_fin(B);  // est: final estimates, then predicted ones
    DevBuf<int32_t> cols_d(B), jn_d(B), fin(B);
    ArnoldiState AS{Hr.p, H.p, hp.p, cs.p, sn.p, gv.p, coef.p, nu.p, est.p, est.p + B,
                    r_fin.p, fin.p, m, kmax};
    LSPR_HIP(hipMemsetAsync(x, 0, B * nvec * sizeof(double2), s));

    SolveResult res;
    res.iters.assign(B, 0);
    res.rel_resid.assign(B, 0.0);
    std::vector<int32_t> jn(B, 0);
    std::vector<double> bnorm(B), nrm_h(B);
    const bool lead = prec == LSPR_FP32_LEAD64;
    const double lead_level = gm.inner_tol > 0.0 ? gm.inner_tol : 0.3;
    std::vector<double> level(B, 1.0);  // latest relative residual estimate per column
    // the two estimates of every column come back through pinned memory in one copy per step
    double* est_h = pinned_estimates(2 * B);
    const double* ef_h = est_h;
    const double* ep_h = est_h + B;

    std::vector<int32_t> cols_now;  // the list cols_d holds
    auto upload_cols = [&](const std::vector<int32_t>& c) {
        if (c == cols_now) return;
        pinned_cols().upload(cols_d.p, c, s);
        cols_now = c;
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
    // inner products of step j (nq final vectors, provisional vector in slot nq) for the columns
    // in cols_d, then the per-column finishing kernel
    // w = A M^{-1} V_j for the listed columns; with LSPR_FP32_LEAD64 in FP64 for the columns
    // whose residual estimate is above the level, in FP32 for the others
    auto product = [&](int j, const std::vector<int32_t>& c) {
        upload_cols(c);
        const int ns = static_cast<int>(c.size());
        // the preconditioner is applied inside the product (packing and row combination)
        const double2* vin = V.p + j * nvec;
        const int64_t vin_stride = m1 * nvec;
        if (!lead) {
            system_apply(g, prec, ns, ratio_d, vin, vin_stride, w.p, nvec, cols_d.p, s, pre);
            return;
        }
        std::vector<int32_t> hi, lo;
        for (int b : c) (level[b] > lead_level ? hi : lo).push_back(b);
        for (int h = 0; h < 2; ++h) {
            const std::vector<int32_t>& part_c = h == 0 ? hi : lo;
            if (part_c.empty()) continue;
            upload_cols(part_c);
            system_apply(g, h == 0 ? LSPR_FP64 : LSPR_FP32, static_cast<int>(part_c.size()),
                         ratio_d, vin, vin_stride, w.p, nvec, cols_d.p, s, pre);
        }
    };
    Event est_ready;
    auto reduce_finish = [&](int ns, int nq, int with_w, int mode, int j) {
        if (with_w)
            hipLaunchKernelGGL(k_dcgs_red<1>, dim3(nblk, ns), dim3(GT), 0, s, V.p, m1, nvec, nq,
                               w.p, cols_d.p, part.p, kmax, nparts);
        else
            hipLaunchKernelGGL(k_dcgs_red<0>, dim3(nblk, ns), dim3(GT), 0, s, V.p, m1, nvec, nq,
                               w.p, cols_d.p, part.p, kmax, nparts);
        hipLaunchKernelGGL(k_dcgs_finish, dim3(ns), dim3(FT),
                           (kmax + 2 * (m1 + 1) + 2 * m + (m1 + 1)) * sizeof(double2), s, part.p,
                           nparts, cols_d.p, mode, j, AS);
        LSPR_HIP(hipGetLastError());
    };
    while (!active.empty()) {
        // ---------------- one restart cycle over the active columns
        std::vector<int32_t> running = active;
        bool queued = false;  // the product of step j is already queued for running's columns
        for (int b : active) jn[b] = 0;
        LSPR_HIP(hipMemsetAsync(fin.p, 0xff, B * sizeof(int32_t), s));  // no final column yet
        for (int j = 0; j < m && !running.empty(); ++j) {
            if (!queued) product(j, running);
            upload_cols(running);
            const int ns = static_cast<int>(running.size());
            {
                // one pass reading j basis vectors, p and w; one reading them again and writing
                // two vectors
                prof::Scope sc("arnoldi", s, 32.0 * (j + 1) * double(nvec) * ns,
                               (2.0 * j + 8.0) * 16.0 * double(nvec) * ns);
                reduce_finish(ns, j, 1, 0, j);
                hipLaunchKernelGGL(k_dcgs_update, dim3(nblk, ns), dim3(GT),
                                   2 * j * sizeof(double2), s, V.p, m1, nvec, j, w.p, cols_d.p,
                                   coef.p, kmax);
                LSPR_HIP(hipGetLastError());
            }
            LSPR_HIP(hipMemcpyAsync(est_h, est.p, 2 * B * sizeof(double), hipMemcpyDeviceToHost, s));
            // The next step's product for the same columns is queued behind the estimates when
            // its precision cannot change (a column's estimate does not rise within a cycle),
            // so the device computes it while the host reads the estimates.  Columns that
            // then finish were multiplied for nothing; the others find w ready.
            // Not queued either when every column is about to finish (estimates within twice the
            // tolerance): that product would be wasted whole.
            queued = j + 1 < m;
            if (lead)
                for (int b : running) queued = queued && level[b] <= lead_level;
            {
                bool all_near = true;
                for (int b : running) all_near = all_near && level[b] <= 2.0 * gm.tol;
                queued = queued && !all_near;
            }
            if (queued) {
                LSPR_HIP(hipEventRecord(est_ready.e, s));
                product(j + 1, running);
                LSPR_HIP(hipEventSynchronize(est_ready.e));
            } else {
                LSPR_HIP(hipStreamSynchronize(s));
            }
            std::vector<int32_t> still, cand;
            for (int b : running) {
                res.iters[b] += 1;
                level[b] = (j >= 1 ? std::min(ef_h[b], ep_h[b]) : ep_h[b]) / bnorm[b];
                if (j >= 1 && ef_h[b] <= gm.tol * bnorm[b]) {
                    jn[b] = j;  // dimension j already meets the tolerance
                    continue;
                }
                const bool last = res.iters[b] >= gm.max_iter || j + 1 == m;
                if (last || ep_h[b] <= gm.tol * bnorm[b]) cand.push_back(b);
                else still.push_back(b);
            }
            if (!cand.empty()) {
                // finalise column j of the candidates: inner products of slot j + 1 alone
                upload_cols(cand);
                const int nc = static_cast<int>(cand.size());
                {
                    prof::Scope sc("arnoldi", s, 8.0 * (j + 1) * double(nvec) * nc,
                                   (j + 2.0) * 16.0 * double(nvec) * nc);
                    reduce_finish(nc, j + 1, 0, 1, j);
                }
                LSPR_HIP(hipMemcpyAsync(est_h, est.p, B * sizeof(double), hipMemcpyDeviceToHost, s));
                LSPR_HIP(hipStreamSynchronize(s));
                for (int b : cand) {
                    jn[b] = j + 1;
                    const bool last = res.iters[b] >= gm.max_iter || j + 1 == m;
                    if (!last && ef_h[b] > gm.tol * bnorm[b]) still.push_back(b);
                }
                std::sort(still.begin(), still.end());
            }
            running.swap(still);
        }
        // ---------------- solution update x += M^{-1} V y and true residual
        upload_cols(active);
        const int ns = static_cast<int>(active.size());
        LSPR_HIP(hipMemcpyAsync(jn_d.p, jn.data(), B * 4, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_backsolve, dim3(ns), dim3(64), (m + 1) * sizeof(double2), s, H.p,
                           gv.p, jn_d.p, cols_d.p, m, y.p);
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
        system_apply(g, lead ? LSPR_FP32 : prec, ns, ratio_d, x, nvec, w.p, nvec, cols_d.p, s);
        hipLaunchKernelGGL(k_resid, dim3(nblk, ns), dim3(GT), 0, s, bvec.p, w.p, V.p, m1 * nvec,
                           nvec, cols_d.p);
        LSPR_HIP(hipGetLastError());
        norms(V.p, m1 * nvec, active);
        std::vector<int32_t> cont;
        for (int b : active) {
            res.rel_resid[b] = nrm_h[b] / bnorm[b];
            level[b] = res.rel_resid[b];
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
