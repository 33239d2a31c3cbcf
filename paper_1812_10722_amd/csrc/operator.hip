// Block matrix-vector product of the discretised single- and double-layer operators
// (Eq. layers_disc with the matrix entries of Eq. layers_element), evaluated as an N-body sum
// with Gauss nodes as sources and panel centroids as targets, accelerated by a treecode
// (section "Acceleration strategies").  All wavelengths of a batch share every launch: the
// real operators act on many real columns at once (the paper's real/imaginary split,
// section "Code modifications and added features", extended to a batch).
//
// Kernels (one launch each per product):
//   k_p2m   box moments of every expanded box, straight from its panels;
//   k_far   per group of 64 consecutive targets: expansions of accepted boxes (M2P) and the
//           direct far-rule sum over the remaining source panels (P2P), compensated;
//   k_near  fine-rule minus far-rule corrections of near-singular pairs and the singular
//           self-term, in FP64.
// Sums are raw: no 1/(4 pi) factor.
#include <cmath>

#include "expansion.hpp"
#include "operator.hpp"
#include "profile.hpp"

namespace lspr {

namespace {

constexpr int NT = 64;   // targets per chunk = wavefront width

// source panels per direct-sum tile (keeps the LDS tiles of k_far under 64 KiB)
template <class T> constexpr int tile_panels() { return sizeof(T) == 8 ? 16 : 32; }

template <class T> __device__ __forceinline__ T rsqrt_t(T x);
template <> __device__ __forceinline__ float rsqrt_t<float>(float x) { return rsqrtf(x); }
template <> __device__ __forceinline__ double rsqrt_t<double>(double x) { return 1.0 / sqrt(x); }

// Knuth's TwoSum: hi + lo += part exactly up to the final rounding.
template <class T>
__device__ __forceinline__ void two_sum_add(T& hi, T& lo, T part) {
    const T s = hi + part;
    const T bb = s - hi;
    const T err = (hi - (s - bb)) + (part - bb);
    hi = s;
    lo += err;
}

// ------------------------------------------------------------------------------- P2M
// Moments of an expanded box about its centre c, for every real column:
//   K columns: M_k = sum_j phi_j sum_g w_g n_j . grad (y_g - c)^k
//   V columns: M_k = sum_j sigma_j sum_g w_g (y_g - c)^k
// then folded to the (P+1)^2 terms with kz <= 1.  Work items are segments of at most
// P2M_SEG consecutive panels of one box, so that large boxes spread over many workgroups;
// a box made of one segment writes its moments directly, the others write partial moments
// that k_p2m_reduce adds in segment order (deterministic).  Block = 256 columns; the
// per-panel polynomial sums of a tile of panels are staged in LDS and shared by all columns.
constexpr int P2M_THREADS = 256;
template <class T, int P> constexpr int p2m_tile() {
    return (16384 / (2 * Expansion<P>::NF * int(sizeof(T)))) < 1
               ? 1
               : ((16384 / (2 * Expansion<P>::NF * int(sizeof(T)))) > 16
                      ? 16
                      : (16384 / (2 * Expansion<P>::NF * int(sizeof(T)))));
}

template <class T, int P>
__global__ void __launch_bounds__(P2M_THREADS)
k_p2m(const Box* __restrict__ boxes, const P2MSeg* __restrict__ segs,
      const double* __restrict__ cen, const T* __restrict__ src, int K,
      const T* __restrict__ dens, int pad, T* __restrict__ mom, T* __restrict__ part) {
    using E = Expansion<P>;
    constexpr E ex{};
    constexpr int NF = E::NF;
    constexpr int P2M_TILE = p2m_tile<T, P>();
    __shared__ T pw[P2M_TILE][8][3][P + 1];      // powers of (y_g - c) per node (K <= 8)
    __shared__ T poly[P2M_TILE][2][NF];           // [0]: V polynomial, [1]: K polynomial
    const P2MSeg sg = segs[blockIdx.x];
    const Box B = boxes[sg.box];
    const int col = blockIdx.y * P2M_THREADS + threadIdx.x;
    const int ncols = 2 * pad;
    const bool kcol = col < pad;
    T acc[NF];
#pragma unroll
    for (int t = 0; t < NF; ++t) acc[t] = T(0);
    const int rs = 4 + 4 * K;
    for (int p0 = sg.start; p0 < sg.end; p0 += P2M_TILE) {
        const int np = min(P2M_TILE, sg.end - p0);
        // powers of node offsets from the box centre
        for (int e = threadIdx.x; e < np * K; e += P2M_THREADS) {
            const int pp = e / K, gq = e % K;
            const int j = p0 + pp;
            const T* r = src + static_cast<size_t>(j) * rs;
            const T d[3] = {static_cast<T>(cen[3 * j] - B.cx) + r[4 + 4 * gq],
                            static_cast<T>(cen[3 * j + 1] - B.cy) + r[5 + 4 * gq],
                            static_cast<T>(cen[3 * j + 2] - B.cz) + r[6 + 4 * gq]};
            for (int a = 0; a < 3; ++a) {
                T v = T(1);
                for (int q = 0; q <= P; ++q) {
                    pw[pp][gq][a][q] = v;
                    v *= d[a];
                }
            }
        }
        __syncthreads();
        // per-panel polynomial sums
        for (int e = threadIdx.x; e < np * NF; e += P2M_THREADS) {
            const int pp = e / NF, t = e % NF;
            const int j = p0 + pp;
            const T* r = src + static_cast<size_t>(j) * rs;
            const int kx = ex.fx[t], ky = ex.fy[t], kz = ex.fz[t];
            T pv = T(0), pk = T(0);
            for (int gq = 0; gq < K; ++gq) {
                const T w = r[7 + 4 * gq];
                const T X = pw[pp][gq][0][kx], Y = pw[pp][gq][1][ky], Z = pw[pp][gq][2][kz];
                pv += w * X * Y * Z;
                T gsum = T(0);
                if (kx > 0) gsum += r[0] * T(kx) * pw[pp][gq][0][kx - 1] * Y * Z;
                if (ky > 0) gsum += r[1] * T(ky) * X * pw[pp][gq][1][ky - 1] * Z;
                if (kz > 0) gsum += r[2] * T(kz) * X * Y * pw[pp][gq][2][kz - 1];
                pk += w * gsum;
            }
            poly[pp][0][t] = pv;
            poly[pp][1][t] = pk;
        }
        __syncthreads();
        if (col < ncols) {
            const int which = kcol ? 1 : 0;
            for (int pp = 0; pp < np; ++pp) {
                const T dj = dens[static_cast<size_t>(p0 + pp) * ncols + col];
#pragma unroll
                for (int t = 0; t < NF; ++t) acc[t] += dj * poly[pp][which][t];
            }
        }
        __syncthreads();
    }
    if (col >= ncols) return;
    // fold the kz >= 2 terms onto kz <= 1 (harmonicity of the kernel)
#pragma unroll
    for (int f = 0; f < E::NFOLD; ++f) {
        acc[ex.fdx[f]] += T(ex.fcx[f]) * acc[ex.fsrc[f]];
        acc[ex.fdy[f]] += T(ex.fcy[f]) * acc[ex.fsrc[f]];
    }
    T* out = sg.slot < 0 ? mom + static_cast<size_t>(sg.box) * E::NR * ncols
                         : part + static_cast<size_t>(sg.slot) * E::NR * ncols;
#pragma unroll
    for (int q = 0; q < E::NR; ++q) out[static_cast<size_t>(q) * ncols + col] = acc[ex.rfull[q]];
}

// mom[box] = sum of its segments' partial moments, in segment order.
template <class T>
__global__ void k_p2m_reduce(const P2MRed* __restrict__ red, int n_red, int nr, int ncols,
                             const T* __restrict__ part, T* __restrict__ mom) {
    const int64_t per = static_cast<int64_t>(nr) * ncols;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= per * n_red) return;
    const int r = static_cast<int>(t / per);
    const int64_t e = t % per;
    const P2MRed R = red[r];
    T s = T(0);
    for (int k = R.slot0; k < R.slot1; ++k) s += part[static_cast<int64_t>(k) * per + e];
    mom[static_cast<int64_t>(R.box) * per + e] = s;
}

// ------------------------------------------------------------------------------- far field
// One block per chunk of up to 64 consecutive targets of one surface; 64 * (pad / CPT)
// threads: lane = target, wavefront = a group of CPT K columns and the matching CPT V columns.
// Own-surface entries come first in both lists, so the own-surface sums are stored before the
// other surfaces are added.
template <class T, int P, int CPT>
__global__ void __launch_bounds__(1024)
k_far(const Chunk* __restrict__ chunks, const Box* __restrict__ boxes,
      const int32_t* __restrict__ m2p_off, const int32_t* __restrict__ m2p_box,
      const int32_t* __restrict__ m2p_self, const int32_t* __restrict__ p2p_off,
      const Range* __restrict__ p2p_rng, const int32_t* __restrict__ p2p_self,
      const double* __restrict__ cen, const T* __restrict__ src, int K,
      const T* __restrict__ dens, const T* __restrict__ mom, int pad,
      double* __restrict__ out_self, double* __restrict__ out_all) {
    using E = Expansion<P>;
    constexpr int NR = E::NR;
    constexpr int PT = tile_panels<T>();
    __shared__ T coef[NR][NT];
    __shared__ T kv_s[PT][NT];
    __shared__ T kk_s[PT][NT];
    const int lane = threadIdx.x % NT;
    const int cc = threadIdx.x / NT;
    const int ncc = blockDim.x / NT;
    const int ncols = 2 * pad;
    const Chunk C = chunks[blockIdx.x];
    const int i = C.start + lane;
    const bool valid = i < C.end;
    const double x0 = valid ? cen[3 * i] : 0.0;
    const double x1 = valid ? cen[3 * i + 1] : 0.0;
    const double x2 = valid ? cen[3 * i + 2] : 0.0;
    const int ck = cc * CPT;       // first K column of this thread
    const int cv = pad + cc * CPT; // first V column

    T hk[CPT], lk[CPT], hv[CPT], lv[CPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) hk[c] = lk[c] = hv[c] = lv[c] = T(0);

    const int m_beg = m2p_off[blockIdx.x], m_end = m2p_off[blockIdx.x + 1];
    const int m_mid = m_beg + m2p_self[blockIdx.x];
    const int p_beg = p2p_off[blockIdx.x], p_end = p2p_off[blockIdx.x + 1];
    const int p_mid = p_beg + p2p_self[blockIdx.x];
    const int rs = 4 + 4 * K;

    for (int phase = 0; phase < 2; ++phase) {
        const int ma = phase == 0 ? m_beg : m_mid, mb = phase == 0 ? m_mid : m_end;
        const int pa = phase == 0 ? p_beg : p_mid, pb = phase == 0 ? p_mid : p_end;
        // ---- expansions of accepted boxes
        for (int e = ma; e < mb; ++e) {
            const int bi = m2p_box[e];
            if (threadIdx.x < NT) {
                const Box B = boxes[bi];
                T F[NR];
                taylor_coefficients<T, P>(static_cast<T>(B.cx - x0), static_cast<T>(B.cy - x1),
                                          static_cast<T>(B.cz - x2), F);
#pragma unroll
                for (int q = 0; q < NR; ++q) coef[q][lane] = valid ? F[q] : T(0);
            }
            __syncthreads();
            const T* M = mom + static_cast<size_t>(bi) * NR * ncols;
            T pk[CPT], pv[CPT];
#pragma unroll
            for (int c = 0; c < CPT; ++c) pk[c] = pv[c] = T(0);
            for (int q = 0; q < NR; ++q) {
                const T f = coef[q][lane];
                const T* mq = M + static_cast<size_t>(q) * ncols;
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    pk[c] += f * mq[ck + c];
                    pv[c] += f * mq[cv + c];
                }
            }
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                two_sum_add(hk[c], lk[c], pk[c]);
                two_sum_add(hv[c], lv[c], pv[c]);
            }
            __syncthreads();
        }
        // ---- direct far-rule sums
        for (int e = pa; e < pb; ++e) {
            const Range R = p2p_rng[e];
            for (int p0 = R.start; p0 < R.end; p0 += PT) {
                const int np = min(PT, R.end - p0);
                for (int pp = cc; pp < PT; pp += ncc) {
                    const int j = p0 + pp;
                    T kv = T(0), kk = T(0);
                    if (valid && pp < np && j != i) {
                        const T* r = src + static_cast<size_t>(j) * rs;
                        const T dx = static_cast<T>(x0 - cen[3 * j]);
                        const T dy = static_cast<T>(x1 - cen[3 * j + 1]);
                        const T dz = static_cast<T>(x2 - cen[3 * j + 2]);
                        const T s = r[0] * dx + r[1] * dy + r[2] * dz;  // height above the plane
                        T sv = T(0), sk = T(0);
                        for (int gq = 0; gq < K; ++gq) {
                            const T ex_ = dx - r[4 + 4 * gq];
                            const T ey_ = dy - r[5 + 4 * gq];
                            const T ez_ = dz - r[6 + 4 * gq];
                            const T w = r[7 + 4 * gq];
                            const T ri = rsqrt_t<T>(ex_ * ex_ + ey_ * ey_ + ez_ * ez_);
                            sv += w * ri;
                            sk += w * ri * ri * ri;
                        }
                        kv = sv;
                        kk = s * sk;
                    }
                    kv_s[pp][lane] = kv;
                    kk_s[pp][lane] = kk;
                }
                __syncthreads();
                T pk[CPT], pv[CPT];
#pragma unroll
                for (int c = 0; c < CPT; ++c) pk[c] = pv[c] = T(0);
                for (int pp = 0; pp < np; ++pp) {
                    const T a = kk_s[pp][lane], b = kv_s[pp][lane];
                    const T* dj = dens + static_cast<size_t>(p0 + pp) * ncols;
#pragma unroll
                    for (int c = 0; c < CPT; ++c) {
                        pk[c] += a * dj[ck + c];
                        pv[c] += b * dj[cv + c];
                    }
                }
#pragma unroll
                for (int c = 0; c < CPT; ++c) {
                    two_sum_add(hk[c], lk[c], pk[c]);
                    two_sum_add(hv[c], lv[c], pv[c]);
                }
                __syncthreads();
            }
        }
        double* o = phase == 0 ? out_self : out_all;
        if (o != nullptr && valid) {
            double* row = o + static_cast<size_t>(i) * ncols;
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                row[ck + c] = static_cast<double>(hk[c]) + static_cast<double>(lk[c]);
                row[cv + c] = static_cast<double>(hv[c]) + static_cast<double>(lv[c]);
            }
        }
    }
}

// ------------------------------------------------------------------------------- near field
// out[i][c] += sum over near-singular pairs (fine - far) * density, plus the singular V_ii,
// split into own-surface and all-surface sums.  Thread = (target, column), FP64.
template <class T>
__global__ void k_near_corr(const int64_t* __restrict__ off, const int32_t* __restrict__ col,
                            const double* __restrict__ dv, const double* __restrict__ dk,
                            const double* __restrict__ vself, const int32_t* __restrict__ surf,
                            int N, const T* __restrict__ dens, int pad,
                            double* __restrict__ out_self, double* __restrict__ out_all) {
    const int ncols = 2 * pad;
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(N) * ncols) return;
    const int i = static_cast<int>(t / ncols), c = static_cast<int>(t % ncols);
    const bool kc = c < pad;
    const int si = surf[i];
    double own = 0.0, other = 0.0;
    for (int64_t e = off[i]; e < off[i + 1]; ++e) {
        const int j = col[e];
        const double v = (kc ? dk[e] : dv[e]) * static_cast<double>(dens[static_cast<size_t>(j) * ncols + c]);
        if (surf[j] == si) own += v;
        else other += v;
    }
    if (!kc) own += vself[i] * static_cast<double>(dens[static_cast<size_t>(i) * ncols + c]);
    out_all[t] += own + other;
    if (out_self != nullptr) out_self[t] += own;
}

template <class T, int P, int CPT>
void launch_far_p(Geometry& g, int pad, const T* dens, const T* mom, double* os, double* oa,
                  hipStream_t s) {
    const int threads = NT * (pad / CPT);
    hipLaunchKernelGGL((k_far<T, P, CPT>), dim3(g.n_chunks), dim3(threads), 0, s, g.chunks.p,
                       g.boxes.p, g.m2p_off.p, g.m2p_box.p, g.m2p_self.p, g.p2p_off.p,
                       g.p2p_rng.p, g.p2p_self.p, g.cen.p, reinterpret_cast<const T*>(g.src.p),
                       g.K, dens, mom, pad, os, oa);
    LSPR_HIP(hipGetLastError());
}

template <class T, int P>
void launch_p2m_p(Geometry& g, int pad, const T* dens, T* mom, hipStream_t s) {
    if (g.n_seg == 0) return;
    const int ncols = 2 * pad;
    const int nr = Expansion<P>::NR;
    T* part = nullptr;
    if (g.n_slots > 0) {
        g.ws_part.reserve(static_cast<size_t>(g.n_slots) * nr * ncols * sizeof(T));
        part = reinterpret_cast<T*>(g.ws_part.p);
    }
    const dim3 grid(g.n_seg, (ncols + P2M_THREADS - 1) / P2M_THREADS);
    hipLaunchKernelGGL((k_p2m<T, P>), grid, dim3(P2M_THREADS), 0, s, g.boxes.p, g.p2m_seg.p,
                       g.cen.p, reinterpret_cast<const T*>(g.src.p), g.K, dens, pad, mom, part);
    LSPR_HIP(hipGetLastError());
    if (g.n_red > 0) {
        const int64_t tot = static_cast<int64_t>(g.n_red) * nr * ncols;
        hipLaunchKernelGGL(k_p2m_reduce<T>, dim3((tot + 255) / 256), dim3(256), 0, s,
                           g.p2m_red.p, g.n_red, nr, ncols, part, mom);
        LSPR_HIP(hipGetLastError());
    }
}

template <class T, int CPT>
void launch_far_cpt(Geometry& g, int pad, const T* dens, const T* mom, double* os, double* oa,
                    hipStream_t s) {
    switch (g.P) {
        case 2: launch_far_p<T, 2, CPT>(g, pad, dens, mom, os, oa, s); break;
        case 4: launch_far_p<T, 4, CPT>(g, pad, dens, mom, os, oa, s); break;
        case 6: launch_far_p<T, 6, CPT>(g, pad, dens, mom, os, oa, s); break;
        case 8: launch_far_p<T, 8, CPT>(g, pad, dens, mom, os, oa, s); break;
        case 10: launch_far_p<T, 10, CPT>(g, pad, dens, mom, os, oa, s); break;
        default: throw Error(LSPR_E_INVALID, "expansion order must be 2, 4, 6, 8 or 10");
    }
}

template <class T>
void apply_far_t(Geometry& g, const Cols& c, const T* dens, double* os, double* oa,
                 hipStream_t s) {
    const double nc = c.ncol;                     // used real columns per operator
    const double esz = sizeof(T);
    const double dens_bytes = double(g.N) * 2 * c.pad * esz;
    const double out_bytes = double(g.N) * 2 * c.pad * 8 * (os ? 2 : 1);
    const int NF = (g.P + 1) * (g.P + 2) * (g.P + 3) / 6;
    const double mom_bytes = double(g.mom_boxes.size()) * g.n_terms * 2 * c.pad * esz;
    T* mom = nullptr;
    if (!g.mom_boxes.empty()) {
        const size_t need = static_cast<size_t>(g.n_boxes) * g.n_terms * 2 * c.pad * sizeof(T);
        g.ws_mom.reserve(need);
        mom = reinterpret_cast<T*>(g.ws_mom.p);
        // per panel of an expanded box: node polynomials (V and K) and the contraction with
        // every used column
        prof::Scope sc("p2m", s, double(g.mom_panels) * (8.0 * g.K * NF + 2.0 * NF * 2 * nc),
                       double(g.mom_panels) * 2 * c.pad * esz + mom_bytes);
        switch (g.P) {
            case 2: launch_p2m_p<T, 2>(g, c.pad, dens, mom, s); break;
            case 4: launch_p2m_p<T, 4>(g, c.pad, dens, mom, s); break;
            case 6: launch_p2m_p<T, 6>(g, c.pad, dens, mom, s); break;
            case 8: launch_p2m_p<T, 8>(g, c.pad, dens, mom, s); break;
            case 10: launch_p2m_p<T, 10>(g, c.pad, dens, mom, s); break;
            default: throw Error(LSPR_E_INVALID, "expansion order must be 2, 4, 6, 8 or 10");
        }
    }
    {
        // direct pairs: per node 15 flops (difference, r^2, rsqrt, two weighted sums), 9 per
        // pair (centroid difference, plane height, product), then 2 flops per used column of
        // each operator; expansion pairs: about 10 flops per coefficient of the recurrence and
        // 2 per coefficient and used column of each operator
        const double f = double(g.p2p_pairs) * (15.0 * g.K + 9.0 + 4.0 * nc) +
                         double(g.m2p_pairs) * (10.0 * g.n_terms + 4.0 * nc * g.n_terms);
        prof::Scope sc("far", s, f, dens_bytes + mom_bytes + out_bytes,
                       (double(g.p2p_pairs) * g.K + double(g.m2p_pairs)) * (nc / 2));
        switch (c.cpt) {
            case 2: launch_far_cpt<T, 2>(g, c.pad, dens, mom, os, oa, s); break;
            case 4: launch_far_cpt<T, 4>(g, c.pad, dens, mom, os, oa, s); break;
            case 16: launch_far_cpt<T, 16>(g, c.pad, dens, mom, os, oa, s); break;
            default: throw Error(LSPR_E_INVALID, "unsupported column blocking");
        }
    }
    const int64_t tot = static_cast<int64_t>(g.N) * 2 * c.pad;
    prof::Scope sc("near", s, double(g.n_near + g.N) * 2.0 * 2 * nc,
                   double(g.n_near) * 20 + dens_bytes + 2 * out_bytes);
    hipLaunchKernelGGL(k_near_corr<T>, dim3((tot + 255) / 256), dim3(256), 0, s,
                       g.near_off64.p, g.near_col.p, g.near_dv.p, g.near_dk.p, g.vself.p,
                       g.surf.p, g.N, dens, c.pad, os, oa);
    LSPR_HIP(hipGetLastError());
}

}  // namespace

Cols make_cols(int ncol) {
    Cols c;
    c.ncol = ncol;
    c.cpt = ncol <= 2 ? 2 : (ncol <= 4 ? 4 : 16);
    c.pad = (ncol + c.cpt - 1) / c.cpt * c.cpt;
    LSPR_REQUIRE(c.pad / c.cpt * NT <= 1024, LSPR_E_INVALID,
                 "too many columns in one product (at most 256 wavelengths)");
    return c;
}

int expansion_terms(int P) { return (P + 1) * (P + 1); }

void apply_raw(Geometry& g, const Cols& c, const void* dens, double* out_self, double* out_all,
               hipStream_t s) {
    double* os = g.S > 1 ? out_self : nullptr;
    if (g.precision == LSPR_FP32)
        apply_far_t<float>(g, c, static_cast<const float*>(dens), os, out_all, s);
    else
        apply_far_t<double>(g, c, static_cast<const double*>(dens), os, out_all, s);
}

}  // namespace lspr
