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
#include <algorithm>
#include <functional>
#include <mutex>
#include <type_traits>
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
// FP64: the hardware estimate (about 23 correct bits) refined by two Newton steps
// y <- y + y (1 - x y^2) / 2, each of which about doubles the correct bits (to within 1-2 ulp),
// instead of a square root followed by a division
template <> __device__ __forceinline__ double rsqrt_t<double>(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
}

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
    T* out = sg.slot < 0 ? mom + static_cast<size_t>(sg.mslot) * E::NR * ncols
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
    mom[static_cast<int64_t>(R.mslot) * per + e] = s;
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
      const T* __restrict__ dens, const T* __restrict__ mom, const int32_t* __restrict__ mom_slot,
      int pad, double* __restrict__ out_self, double* __restrict__ out_all) {
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
            const T* M = mom + static_cast<size_t>(mom_slot[bi]) * NR * ncols;
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

// ------------------------------------------------------------------------------- far field, MFMA
// Far-field sums on matrix cores, FP32 or FP64.  For a chunk of 64 targets every interaction is
// a small dense product: an expansion is (64 x terms) . (terms x columns) of Taylor
// coefficients and box moments, a direct tile is (64 x panels) . (panels x columns) of
// far-rule kernel values and densities.  The left factors depend on geometry only; build_tiles
// stores them once per geometry, in the operand order of v_mfma_{f32,f64}_16x16x4 (lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; see out_row for the result rows): for
// K-step s and lane l, the four target tiles' values are four consecutive elements.  The product
// then streams those tiles from HBM and spends its time in matrix-core instructions.  In FP32
// each tile's product is accumulated by the matrix cores and then added to an FP64 running sum
// per output, so rounding does not grow with the number of tiles; in FP64 the matrix cores
// accumulate every tile directly.
typedef float v4f __attribute__((ext_vector_type(4)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

// Direct tiles: a chunk's direct-sum range is cut into pieces of up to 4 direct_steps()
// source panels, one tile each (K-steps = panels / 4 rounded up).  That is the length of an
// expansion slice (at least DSTEPS), so every tile covers the prefetch of the next one for as
// long and the kernels run one loop of that many steps for both kinds; each tile's partial is
// summed in FP32 by the matrix cores before it joins the FP64 running sum.
constexpr int DSTEPS = 8;

// Expansion tiles of high orders are cut along the Taylor terms into slices of equal K-steps
// (at most 21, the P = 8 tile), each a tile of its own with its slice of moment rows; orders up
// to 10 keep one tile per expansion.  The kernels then never stage or hold more than one slice.
constexpr int expansion_slices(int n_terms) {
    const int steps = (n_terms + 3) / 4;
    return steps <= 31 ? 1 : (steps + 20) / 21;
}
constexpr int expansion_slice_steps(int n_terms) {
    const int steps = (n_terms + 3) / 4, n = expansion_slices(n_terms);
    return (steps + n - 1) / n;
}
constexpr int direct_steps(int n_terms) {
    return expansion_slice_steps(n_terms) > DSTEPS ? expansion_slice_steps(n_terms) : DSTEPS;
}

// Element of a tile's left factor (within one factor) holding K-step st, lane l (row 16 g + r
// of the step's 16 x 4 operand: l = 16 g + r) and target tile mt.  FP32: the four target tiles
// of a lane and step are adjacent (16 bytes, one 128-bit read).  FP64: the 32 bytes are split
// into two planes of 64 lanes per step (target tiles 0-1, then 2-3), so that both 128-bit reads
// of a step, and the copies that stage it, are contiguous across the lanes.
template <class T>
__host__ __device__ __forceinline__ size_t tile_index(int st, int l, int mt) {
    if constexpr (sizeof(T) == 4)
        return (static_cast<size_t>(st) * 64 + l) * 4 + mt;
    else
        return (static_cast<size_t>(2 * st + (mt >> 1)) * 64 + l) * 2 + (mt & 1);
}

template <class T>
struct alignas(4 * sizeof(T)) Quad {
    T x, y, z, w;
};

template <class T>
struct Mma;
template <>
struct Mma<float> {
    using acc = v4f;
    static __device__ __forceinline__ v4f op(float a, float b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct Mma<double> {
    using acc = v4d;
    static __device__ __forceinline__ v4d op(double a, double b, v4d c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// Row within a 16 x 16 result tile of accumulator element q of lane group grp = lane / 16:
// v_mfma_f32_16x16x4f32 holds rows 4 grp + q, v_mfma_f64_16x16x4f64 rows grp + 4 q.
template <class T>
__device__ __forceinline__ int out_row(int grp, int q) {
    return sizeof(T) == 4 ? 4 * grp + q : grp + 4 * q;
}

// Scalar offset of the next K-step's B operand.  The empty asm makes each step's offset opaque,
// so that the compiler forms it with one scalar add instead of keeping every step's offset in
// its own scalar register across the tile loop.
__device__ __forceinline__ uint32_t next_step(uint32_t so, uint32_t step) {
    so += step;
    asm volatile("" : "+s"(so));
    return so;
}

// Buffer resource over [p, p + bytes) for raw buffer loads: out-of-range offsets read zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, bytes, 0x00020000);
}

// One element of a raw buffer load (out-of-range offsets read zero).
template <class T>
__device__ __forceinline__ T load_elem(__amdgpu_buffer_rsrc_t rb, uint32_t voff, uint32_t soff);
template <>
__device__ __forceinline__ float load_elem<float>(__amdgpu_buffer_rsrc_t rb, uint32_t voff,
                                                  uint32_t soff) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rb, voff, soff, 0));
}
template <>
__device__ __forceinline__ double load_elem<double>(__amdgpu_buffer_rsrc_t rb, uint32_t voff,
                                                    uint32_t soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rb, voff, soff, 0));
}

// Left factors in LDS, in the store's order (tile_index): a K-step's operand of one lane is
// one 128-bit read in FP32 and one from each of the step's two planes in FP64, both
// conflict-free.
template <class T>
__device__ __forceinline__ Quad<T> lds_quad(const float4* ab, int st, int lane) {
    if constexpr (sizeof(T) == 4) {
        return reinterpret_cast<const Quad<float>*>(ab)[st * 64 + lane];
    } else {
        const float4 lo = ab[2 * st * 64 + lane], hi = ab[(2 * st + 1) * 64 + lane];
        Quad<double> q;
        q.x = __builtin_bit_cast(double, make_float2(lo.x, lo.y));
        q.y = __builtin_bit_cast(double, make_float2(lo.z, lo.w));
        q.z = __builtin_bit_cast(double, make_float2(hi.x, hi.y));
        q.w = __builtin_bit_cast(double, make_float2(hi.z, hi.w));
        return q;
    }
}

// Far field on matrix cores, one operator per workgroup (FP32 or FP64 products).  Workgroups b, b + 8, ... handle one chunk (all on
// the same XCD, so the later ones read the chunk's left factors from L2): the double-layer (K)
// and single-layer (V) columns, each in 1 or 2 halves of 4 column groups of 16, one group per
// wave.  Expansion tiles share one left factor between the operators; direct tiles hold the K
// factor and then the V factor.
// Latency hiding, per tile: the next tile's left factor is fetched into registers and stored to
// the single LDS buffer between two barriers at the end of the tile; each B operand of the next
// tile is requested into its register right after the current tile's step has used it; the
// descriptor two tiles ahead comes with the vector loads.  No scalar load and no register spill
// remains in the loop; at P = 8, 128 VGPRs and 21.5 KB of LDS: four workgroups (16 waves) per CU
// (three at P = 10).  FP64: the same scheme on v_mfma_f64_16x16x4f64, whose accumulators are
// the FP64 sums themselves; the left factor takes twice the LDS, three workgroups per CU.
// Narrow products (one or two column groups per operator) split the K-steps instead: S = 4 / G
// waves share each of the G column groups, wave k taking steps k, k + S, ...; at the end their
// FP64 sums are added in wave order through LDS.  S = 1 is the wide kernel.
// OPS = 2: eight waves per workgroup, waves 0-3 on the K columns and 4-7 on the V columns (of
// one column half), so each left factor is staged once for both operators (a direct tile's two
// factors side by side) and a chunk's tiles are read by `halves` workgroups instead of
// 2 * halves; each wave's arithmetic is that of OPS = 1.
template <class T, int NSM, int S, int OPS = 1>
__global__ void __launch_bounds__(256 * OPS,
                                  OPS == 2 ? (sizeof(T) == 8 ? 1 : 2)
                                           : (sizeof(T) == 8 || (S > 1 && NSM > 21) ? 2
                                                                                    : (S > 1 || NSM > 21 ? 3 : 4)))
k_far_tiles_op(const Chunk* __restrict__ chunks, const FarItem* __restrict__ items,
               const int32_t* __restrict__ item_order, const int32_t* __restrict__ tile_self,
               const TileDesc* __restrict__ tiles,
               const T* __restrict__ tileA, const T* __restrict__ dens, const T* __restrict__ mom,
               int pad, int nwc, int halves, double* __restrict__ out_self,
               double* __restrict__ out_all, double* __restrict__ part) {
    static_assert(OPS == 1 || OPS == 2, "one or both operators per workgroup");
    constexpr int NTHR = 256 * OPS;
    constexpr uint32_t ES = sizeof(T);       // bytes per element
    constexpr int EPU = 16 / sizeof(T);      // elements per 16-byte unit
    using Acc = typename Mma<T>::acc;
    extern __shared__ float4 abuf16[];  // the current tile's left factor
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int c16 = lane & 15, grp = lane >> 4;
    const int ncols = 2 * pad;
    // OPS = 1: 2 * halves workgroups per chunk, at b, b + 8, ...: operator j & 1, column half
    // j >> 1.  OPS = 2: halves workgroups per chunk, column half j, operator wave / 4.
    const int b = blockIdx.x;
    const int per = OPS == 2 ? halves : 2 * halves;
    const int j = (b >> 3) % per;
    const int opr = OPS == 2 ? wave >> 2 : j & 1;  // 0: K columns, 1: V columns
    const int hj = OPS == 2 ? j : j >> 1;          // column half
    constexpr int G = 4 / S;                // column groups per workgroup and operator
    // wave-uniform values in scalar registers, so that the branches on them are scalar
    const int kpart = __builtin_amdgcn_readfirstlane((wave & 3) % S);  // share of the K-steps
    const int wg = __builtin_amdgcn_readfirstlane((wave & 3) / S + G * hj);  // column group
    const int item = item_order[(b >> 3) / per * 8 + (b & 7)];
    if (item < 0) return;
    const FarItem I = items[item];
    const int chunk = I.chunk;
    const Chunk C = chunks[chunk];
    const int ntg = C.end - C.start;
    const bool mma = wg < nwc;
    const int col = opr * pad + 16 * wg + c16;  // this lane's column
    // B operand of K-step st: row 4 st + grp of the tile, column col, i.e. byte offset
    // boff + st * bstep from the tile's first row (rows past the tile read zero)
    const uint32_t boff = static_cast<uint32_t>(grp * ncols + (mma ? col : 0)) * ES;
    const uint32_t bstep = 4u * ES * static_cast<uint32_t>(ncols);
    Acc acc[4];
    double run[4][4];  // FP32: FP64 running sums of the tiles' partials
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        acc[a] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 4; ++q) run[a][q] = 0.0;
    }
    // this wave's sum of target row 16 mt + out_row(grp, q) of its column
    auto own = [&](int mt, int q) -> double {
        if constexpr (sizeof(T) == 4) return run[mt][q];
        else return acc[mt][q];
    };
    // a whole chunk writes its own-surface sums after its own-surface tiles and its sums over
    // all surfaces at the end; a piece writes its partial sums to its scratch block (rows from 0)
    const bool whole = I.slot < 0;
    const int t_beg = I.t0, t_end = I.t1;
    const int t_mid = whole ? t_beg + tile_self[chunk] : t_beg;
    double* const o_self = whole ? out_self : nullptr;
    double* const o_all = whole ? out_all + static_cast<size_t>(C.start) * ncols
                                : part + static_cast<size_t>(I.slot) * NT * ncols;
    // Writes the sums (with S > 1 the first wave of each column group adds the others' sums, in
    // wave order, from LDS after the left-factor buffer; all waves call it); out: the chunk's
    // first row.
    auto write_sums = [&](double* out) {
        double sum[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int q = 0; q < 4; ++q) sum[mt][q] = own(mt, q);
        if constexpr (S > 1) {
            // one 8 KB slot per column group (and operator), passed from wave to wave; the slots
            // follow the left-factor buffer
            constexpr int AEL = OPS * (NSM > DSTEPS ? NSM : DSTEPS) * 256;
            double* red = reinterpret_cast<double*>(abuf16 + AEL / EPU) +
                          ((wave & 3) / S + (OPS == 2 ? opr * G : 0)) * 16 * 64;
            for (int k = 1; k < S; ++k) {
                if (kpart == k)
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                        for (int q = 0; q < 4; ++q) red[(4 * mt + q) * 64 + lane] = own(mt, q);
                __syncthreads();
                if (kpart == 0)
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                        for (int q = 0; q < 4; ++q) sum[mt][q] += red[(4 * mt + q) * 64 + lane];
                __syncthreads();
            }
        }
        if (!mma || kpart != 0) return;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = 16 * mt + out_row<T>(grp, q);
                if (t < ntg) out[static_cast<size_t>(t) * ncols + col] = sum[mt][q];
            }
    };
    // B operands: NB values per lane whatever the tile's kind (steps past a tile's rows read
    // zero without touching memory).  Operand st of the next tile is requested into the same
    // register as soon as step st of the current tile has been issued, so the loads of a tile's
    // operands overlap the whole previous tile with one register per step.
    constexpr int NB = NSM > DSTEPS ? NSM : DSTEPS;
    constexpr int NBS = (NB + S - 1) / S;  // operand registers per wave
    auto b_rsrc = [&](const TileDesc& D, uint32_t rows) {
        const T* bsrc = D.kind == 0 ? mom : dens;
        return buffer_rsrc(bsrc + static_cast<size_t>(D.b_row0) * ncols,
                           rows * static_cast<uint32_t>(ncols) * ES);
    };
    auto load_b_at = [&](__amdgpu_buffer_rsrc_t rb, uint32_t so) {
        return load_elem<T>(rb, boff, so);
    };
    auto load_b = [&](__amdgpu_buffer_rsrc_t rb, int st) {
        // the per-step offset is uniform: it goes in the scalar offset, not in a VGPR
        return load_elem<T>(rb, boff, st * bstep);
    };
    // Tile descriptors: the current and next in scalar registers, the one after that
    // requested with the vector prefetch of each tile (one 128-bit load, zero past the chunk's
    // last tile), so no scalar load waits inside the loop.
    const __amdgpu_buffer_rsrc_t rt = buffer_rsrc(tiles + t_beg, static_cast<uint32_t>(t_end - t_beg) * 16u);
    auto to_desc = [](const v4u& w) {
        const uint32_t w0 = __builtin_amdgcn_readfirstlane(w[0]);
        TileDesc D;
        D.kind = static_cast<int16_t>(w0 & 0xffffu);
        D.nstep = static_cast<int16_t>(w0 >> 16);
        D.a_blk = static_cast<int32_t>(__builtin_amdgcn_readfirstlane(w[1]));
        D.b_row0 = static_cast<int32_t>(__builtin_amdgcn_readfirstlane(w[2]));
        D.b_rows = static_cast<int32_t>(__builtin_amdgcn_readfirstlane(w[3]));
        return D;
    };
    // the part of a left factor this workgroup uses: all of an expansion tile, the factor of its
    // own operator of a direct tile, or with OPS = 2 both (its first element, count).  Every
    // tile is staged as NB K-steps (OPS = 2: 2 NB): the loads past its own elements read zero,
    // so the steps a tile does not have add nothing and the loop needs no branch.
    auto own_off = [&](const TileDesc& D) {
        return D.a_off() +
               (OPS == 1 && D.kind == 1 ? static_cast<int64_t>(opr) * D.nstep * 256 : 0);
    };
    auto own_elems = [](const TileDesc& D) {
        return 256 * D.nstep * (OPS == 2 && D.kind == 1 ? 2 : 1);
    };
    constexpr int STAGE16 = OPS * NB * 256 / EPU;  // 16-byte units staged per tile
    TileDesc Te = tiles[t_beg < t_end ? t_beg : 0];
    TileDesc Tn = tiles[t_beg + 1 < t_end ? t_beg + 1 : 0];
    T bc[NBS];
    if (t_beg < t_end) {
        const int n16 = own_elems(Te) / EPU;
        const float4* src = reinterpret_cast<const float4*>(tileA + own_off(Te));
        for (int k = tid; k < STAGE16; k += NTHR)
            abuf16[k] = k < n16 ? src[k] : make_float4(0.f, 0.f, 0.f, 0.f);
        const __amdgpu_buffer_rsrc_t rb = b_rsrc(Te, static_cast<uint32_t>(Te.b_rows));
#pragma unroll
        for (int i = 0; i < NBS; ++i) bc[i] = load_b(rb, kpart + S * i);
    }
    __syncthreads();
    // a left factor is NA elements per thread: NA / EPU 16-byte units at unit index
    // tid + NTHR r, then NA % EPU elements at element index NTHR EPU (NA / EPU) + tid + NTHR r
    constexpr int NA = NB;
    constexpr int QA = NA / EPU, RA = NA % EPU;
    // one tile: prefetches for the next, products of this one (all waves of the workgroup run
    // it together: it ends with a barrier)
    auto tile = [&](int e) {
        // the descriptor two tiles ahead, the next left factor into registers (past the last
        // tile it reads zero and is not stored), and the descriptor of the next B operands
        // (empty past the last tile)
        const v4u dn = __builtin_amdgcn_raw_buffer_load_b128(
            rt, 0, static_cast<uint32_t>(e + 2 - t_beg) * 16u, 0);
        float4 pf[QA];
        T pr[RA > 0 ? RA : 1];
        const bool more = e + 1 < t_end;
        const int n16n = more ? STAGE16 : 0;  // past the tile's own elements: zeros
        {
            const __amdgpu_buffer_rsrc_t ra =
                buffer_rsrc(tileA + own_off(Tn), more ? own_elems(Tn) / EPU * 16u : 0u);
#pragma unroll
            for (int r = 0; r < QA; ++r) {
                const auto v = __builtin_amdgcn_raw_buffer_load_b128(ra, tid * 16, r * NTHR * 16, 0);
                pf[r] = make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]),
                                    __uint_as_float(v[2]), __uint_as_float(v[3]));
            }
#pragma unroll
            for (int r = 0; r < RA; ++r)
                pr[r] = load_elem<T>(ra, tid * ES, (QA * EPU * NTHR + r * NTHR) * ES);
        }
        const __amdgpu_buffer_rsrc_t rbn = b_rsrc(Tn, more ? static_cast<uint32_t>(Tn.b_rows) : 0u);
        // Every wave, with columns or not, issues the same vector loads in the same order, and
        // only the matrix-core blocks are conditional (scalar branches): the wait counts the
        // compiler places before the staging stores then cover the left-factor loads alone, not
        // the B operands just requested for the next tile (on a path that skipped those loads
        // the counts would be too small for the path that made them).
        {
            // with OPS = 2 the V waves read a direct tile's second factor
            const float4* ab = abuf16 + (OPS == 2 && Te.kind == 1 ? opr * Te.nstep * 256 / EPU : 0);
            auto flush = [&]() {
                if constexpr (sizeof(T) == 4) {
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
#pragma unroll
                        for (int q = 0; q < 4; ++q) run[a][q] += static_cast<double>(acc[a][q]);
                        acc[a] = Acc{0, 0, 0, 0};
                    }
                }
            };
            // one loop for every tile: NB steps of LDS reads, products and B prefetches; FP32:
            // each wave's partial of every DSTEPS K-steps of the tile joins the FP64 running
            // sums, so no FP32 partial sums more than 4 DSTEPS panels or terms.  Each step's
            // left operand is read from LDS one step ahead.
            if constexpr (S == 1) {
                // the tile's own steps on the matrix cores (a uniform branch per step), the next
                // tile's operands requested for every step
                const int ns = mma ? Te.nstep : 0;
                uint32_t so = 0;
                Quad<T> a = lds_quad<T>(ab, 0, lane);
#pragma unroll
                for (int st = 0; st < NB; ++st) {
                    Quad<T> an = a;
                    if (st + 1 < NB) an = lds_quad<T>(ab, st + 1, lane);
                    if (st < ns) {
                        acc[0] = Mma<T>::op(a.x, bc[st], acc[0]);
                        acc[1] = Mma<T>::op(a.y, bc[st], acc[1]);
                        acc[2] = Mma<T>::op(a.z, bc[st], acc[2]);
                        acc[3] = Mma<T>::op(a.w, bc[st], acc[3]);
                    }
                    bc[st] = load_b_at(rbn, so);
                    so = next_step(so, bstep);
                    a = an;
                }
                flush();
            } else {
                const int ns = mma ? NB : 0;
                Quad<T> a = lds_quad<T>(ab, kpart < NB ? kpart : NB - 1, lane);
#pragma unroll
                for (int i = 0; i < NBS; ++i) {
                    const int st = kpart + S * i;
                    Quad<T> an = a;
                    if (i + 1 < NBS) an = lds_quad<T>(ab, st + S < NB ? st + S : NB - 1, lane);
                    if (st < ns) {
                        acc[0] = Mma<T>::op(a.x, bc[i], acc[0]);
                        acc[1] = Mma<T>::op(a.y, bc[i], acc[1]);
                        acc[2] = Mma<T>::op(a.z, bc[i], acc[2]);
                        acc[3] = Mma<T>::op(a.w, bc[i], acc[3]);
                    }
                    bc[i] = load_b(rbn, st);
                    a = an;
                    // this wave's steps of K-steps [8 m, 8 m + 8) are i in [8 m / S, 8 (m + 1) / S)
                    if ((i + 1) % (DSTEPS / S) == 0 || i + 1 == NBS) flush();
                }
            }
        }
        __syncthreads();  // every wave is done with this tile's left factor
        {
            float4* dst = abuf16;
#pragma unroll
            for (int r = 0; r < QA; ++r) {
                const int k = tid + r * NTHR;
                if (k < n16n) dst[k] = pf[r];
            }
            T* dst1 = reinterpret_cast<T*>(dst);
#pragma unroll
            for (int r = 0; r < RA; ++r) {
                const int k = QA * EPU * NTHR + tid + r * NTHR;  // element index
                if (k < EPU * n16n) dst1[k] = pr[r];
            }
        }
        Te = Tn;
        Tn = to_desc(dn);
        __syncthreads();
    };
    // own-surface tiles first: their sums are the own-surface result (written between the two
    // loops, so that no output address is kept in registers across the tile loop)
    for (int e = t_beg; e < t_mid; ++e) tile(e);
    if (o_self != nullptr) write_sums(o_self + static_cast<size_t>(C.start) * ncols);
    for (int e = t_mid; e < t_end; ++e) tile(e);
    write_sums(o_all);
}

// FP32 products with the left factors read straight into LDS, one operator's columns per
// eight-wave workgroup: 8 / S column groups of 16, S waves each.  S = 1 (more than 64 columns
// per operator): eight column groups, both column halves, so the tiles of a work item are read
// by two workgroups (the two operators) instead of four.  S = 4, 8 (up to 32, 16 columns): S
// waves share a column group and split its K-steps, wave k taking steps k, k + S, ..., with its
// FP32 partial of each tile (at most 6 K-steps: 24 panels or terms) added to its FP64 sums, and
// the S waves' FP64 sums added in wave order through LDS at the end.
// Three LDS buffers: at the start of tile e every wave requests its share of the left factor of
// tile e + 2 (whole K-steps of 1 KB, by buffer loads that write LDS; zeros past the tile's
// elements) into the buffer tile e - 1 used; at the end each wave waits for its own requests of
// tile e + 1, with everything it has requested since still outstanding, and one barrier ends
// the tile.  For S = 1 the arithmetic per wave is that of k_far_tiles_op<float, NSM, 1> (the
// same B operands, K-step order, FP32 partial per tile and FP64 running sums), so both give the
// same sums.  Two workgroups (16 waves) per CU, each with 3 x 21 KB of LDS at P = 8.
// Requires work items that do not span a chunk's own-surface boundary (plan_items, cut_self).
template <int NSM, int S>
__global__ void __launch_bounds__(512, 2)
k_far_wide(const Chunk* __restrict__ chunks, const FarItem* __restrict__ items,
           const int32_t* __restrict__ item_order, const int32_t* __restrict__ tile_self,
           const TileDesc* __restrict__ tiles, const float* __restrict__ tileA,
           const float* __restrict__ dens, const float* __restrict__ mom, int pad, int nwc,
           double* __restrict__ out_self, double* __restrict__ out_all,
           double* __restrict__ part) {
    static_assert(S == 1 || S == 4 || S == 8, "waves per column group");
    constexpr int NB = NSM > DSTEPS ? NSM : DSTEPS;
    constexpr int NBS = (NB + S - 1) / S;  // K-steps (B operands) per wave and tile
    constexpr int G = 8 / S;               // column groups per workgroup
    constexpr int NREQ = (NB + 7) / 8;     // K-steps each wave requests per tile
    typedef __attribute__((address_space(3))) void* lds_ptr;
    __shared__ float4 lb0[NB * 64];
    __shared__ float4 lb1[NB * 64];
    __shared__ float4 lb2[NB * 64];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wg = wave / S, kpart = wave % S;  // column group, share of the K-steps
    const int c16 = lane & 15, grp = lane >> 4;
    const int ncols = 2 * pad;
    // two workgroups per work item, at b and b + 8: operator (b >> 3) & 1
    const int b = blockIdx.x;
    const int opr = (b >> 3) & 1;
    const int item = item_order[(b >> 4) * 8 + (b & 7)];
    if (item < 0) return;
    const FarItem I = items[item];
    const int chunk = I.chunk;
    const Chunk C = chunks[chunk];
    const int ntg = C.end - C.start;
    const bool mma = wg < nwc;
    const int col = opr * pad + 16 * wg + c16;
    const uint32_t boff = static_cast<uint32_t>(grp * ncols + (mma ? col : 0)) * 4u;
    const uint32_t bstep = 16u * static_cast<uint32_t>(ncols);
    v4f acc[4];
    double run[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        acc[a] = v4f{0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 4; ++q) run[a][q] = 0.0;
    }
    const bool whole = I.slot < 0;
    const int t_beg = I.t0, t_end = I.t1;
    const int t_mid = whole ? t_beg + tile_self[chunk] : t_beg;
    double* const o_self = whole ? out_self : nullptr;
    double* const o_all = whole ? out_all + static_cast<size_t>(C.start) * ncols
                                : part + static_cast<size_t>(I.slot) * NT * ncols;
    // (S > 1: all waves call it; the first wave of each column group adds the others' sums in
    // wave order, through one 8 KB slot per group in the LDS buffers, after every request into
    // them has landed)
    auto write_sums = [&](double* out) {
        double sum[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int q = 0; q < 4; ++q) sum[mt][q] = run[mt][q];
        if constexpr (S > 1) {
            constexpr int SPB = NB * 64 * 16 / (16 * 64 * 8);  // 8 KB slots per buffer
            static_assert(G <= 3 * SPB, "reduction slots");
            float4* const base = wg < SPB ? lb0 : (wg < 2 * SPB ? lb1 : lb2);
            double* red = reinterpret_cast<double*>(base) + (wg % SPB) * 16 * 64;
            __syncthreads();
            for (int k = 1; k < S; ++k) {
                if (kpart == k)
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                        for (int q = 0; q < 4; ++q) red[(4 * mt + q) * 64 + lane] = run[mt][q];
                __syncthreads();
                if (kpart == 0)
#pragma unroll
                    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                        for (int q = 0; q < 4; ++q) sum[mt][q] += red[(4 * mt + q) * 64 + lane];
                __syncthreads();
            }
        }
        if (!mma || kpart != 0) return;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = 16 * mt + out_row<float>(grp, q);
                if (t < ntg) out[static_cast<size_t>(t) * ncols + col] = sum[mt][q];
            }
    };
    auto b_rsrc = [&](const TileDesc& D, uint32_t rows) {
        const float* bsrc = D.kind == 0 ? mom : dens;
        return buffer_rsrc(bsrc + static_cast<size_t>(D.b_row0) * ncols,
                           rows * static_cast<uint32_t>(ncols) * 4u);
    };
    auto to_desc = [](const v4u& w) {
        const uint32_t w0 = __builtin_amdgcn_readfirstlane(w[0]);
        TileDesc D;
        D.kind = static_cast<int16_t>(w0 & 0xffffu);
        D.nstep = static_cast<int16_t>(w0 >> 16);
        D.a_blk = static_cast<int32_t>(__builtin_amdgcn_readfirstlane(w[1]));
        D.b_row0 = static_cast<int32_t>(__builtin_amdgcn_readfirstlane(w[2]));
        D.b_rows = static_cast<int32_t>(__builtin_amdgcn_readfirstlane(w[3]));
        return D;
    };
    // this wave's requests for the left factor of tile D (its own operator's factor of a
    // direct tile): K-steps wave, wave + 8, ... (the last step of the tile may be requested by
    // more than one wave, with the same data), none of the tile's data when `more` is false
    auto request = [&](const TileDesc& D, bool more, float4* L) {
        const int64_t off = D.a_off() + (D.kind == 1 ? static_cast<int64_t>(opr) * D.nstep * 256 : 0);
        const __amdgpu_buffer_rsrc_t ra =
            buffer_rsrc(tileA + off, more ? static_cast<uint32_t>(D.nstep) * 1024u : 0u);
#pragma unroll
        for (int k = 0; k < NREQ; ++k) {
            const int st = wave + 8 * k < NB ? wave + 8 * k : NB - 1;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr)(L + st * 64), 16, lane * 16,
                                                     st * 1024, 0, 0);
        }
    };
    // The work items of these launches never span the own-surface boundary (the plan cuts
    // every chunk there): a whole chunk's own-surface sums are its sums over all its tiles, or
    // zero when it has no own-surface tiles.
    if (o_self != nullptr && t_mid == t_beg) write_sums(o_self + static_cast<size_t>(C.start) * ncols);
    const __amdgpu_buffer_rsrc_t rt =
        buffer_rsrc(tiles + t_beg, static_cast<uint32_t>(t_end - t_beg) * 16u);
    TileDesc Te = tiles[t_beg < t_end ? t_beg : 0];
    TileDesc Tn = tiles[t_beg + 1 < t_end ? t_beg + 1 : 0];
    TileDesc Tnn = tiles[t_beg + 2 < t_end ? t_beg + 2 : 0];
    float bc[NBS];
    {
        request(Te, t_beg < t_end, lb0);
        request(Tn, t_beg + 1 < t_end, lb1);
        const __amdgpu_buffer_rsrc_t rb =
            b_rsrc(Te, t_beg < t_end ? static_cast<uint32_t>(Te.b_rows) : 0u);
#pragma unroll
        for (int i = 0; i < NBS; ++i) bc[i] = load_elem<float>(rb, boff, (kpart + S * i) * bstep);
    }
    __syncthreads();  // waits for every load: the first two left factors are complete
    // one tile: reads buffer P, requests the left factor of tile e + 2 into buffer P + 2
    auto tile = [&](int e, auto par) {
        constexpr int P = decltype(par)::value;
        float4* const Lc = P == 0 ? lb0 : (P == 1 ? lb1 : lb2);
        float4* const Lr = P == 0 ? lb2 : (P == 1 ? lb0 : lb1);
        const v4u dn = __builtin_amdgcn_raw_buffer_load_b128(
            rt, 0, static_cast<uint32_t>(e + 3 - t_beg) * 16u, 0);
        const bool more = e + 1 < t_end;
        request(Tnn, e + 2 < t_end, Lr);
        const __amdgpu_buffer_rsrc_t rbn = b_rsrc(Tn, more ? static_cast<uint32_t>(Tn.b_rows) : 0u);
        const int ns = mma ? Te.nstep : 0;
        auto flush = [&]() {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
#pragma unroll
                for (int r = 0; r < 4; ++r) run[q][r] += static_cast<double>(acc[q][r]);
                acc[q] = v4f{0, 0, 0, 0};
            }
        };
        if constexpr (S == 1) {
            uint32_t so = 0;
            Quad<float> a = lds_quad<float>(Lc, 0, lane);
#pragma unroll
            for (int st = 0; st < NB; ++st) {
                Quad<float> an = a;
                if (st + 1 < NB) an = lds_quad<float>(Lc, st + 1, lane);
                if (st < ns) {
                    acc[0] = Mma<float>::op(a.x, bc[st], acc[0]);
                    acc[1] = Mma<float>::op(a.y, bc[st], acc[1]);
                    acc[2] = Mma<float>::op(a.z, bc[st], acc[2]);
                    acc[3] = Mma<float>::op(a.w, bc[st], acc[3]);
                }
                bc[st] = load_elem<float>(rbn, boff, so);
                so = next_step(so, bstep);
                a = an;
            }
            flush();
        } else {
            Quad<float> a = lds_quad<float>(Lc, kpart < NB ? kpart : NB - 1, lane);
#pragma unroll
            for (int i = 0; i < NBS; ++i) {
                const int st = kpart + S * i;
                Quad<float> an = a;
                if (i + 1 < NBS) an = lds_quad<float>(Lc, st + S < NB ? st + S : NB - 1, lane);
                if (st < ns) {
                    acc[0] = Mma<float>::op(a.x, bc[i], acc[0]);
                    acc[1] = Mma<float>::op(a.y, bc[i], acc[1]);
                    acc[2] = Mma<float>::op(a.z, bc[i], acc[2]);
                    acc[3] = Mma<float>::op(a.w, bc[i], acc[3]);
                }
                bc[i] = load_elem<float>(rbn, boff, st * bstep);
                a = an;
                // (at S >= 4 a wave holds at most 6 K-steps of a tile: its FP32 partial of the
                // tile spans at most 24 panels or terms)
                if (i + 1 == NBS) flush();
            }
        }
        // this wave's requests of tile e + 1 (made at the start of tile e - 1, or before the
        // first tile) are complete when no more than the loads issued after them are
        // outstanding: the NBS B operands of tile e - 1, this tile's descriptor, requests and
        // NBS B operands (vmcnt field split over bits 3:0 and 15:14; expcnt and lgkmcnt not
        // waited for); the barrier then makes every wave's part visible and frees Lc for the
        // next tile's request
        constexpr int VM = 2 * NBS + 1 + NREQ;
        static_assert(VM < 64, "vmcnt range");
        __builtin_amdgcn_s_waitcnt((VM & 15) | (7 << 4) | (15 << 8) | ((VM >> 4) << 14));
        // (the empty statements keep the compiler from moving memory accesses across the
        // barrier, which itself orders none)
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        Te = Tn;
        Tn = Tnn;
        Tnn = to_desc(dn);
    };
    // the buffer a tile reads cycles with its position in the item: three copies of the tile in
    // sequence, so that no branch selects among them
    for (int e = t_beg; e < t_end;) {
        tile(e++, std::integral_constant<int, 0>{});
        if (e >= t_end) break;
        tile(e++, std::integral_constant<int, 1>{});
        if (e >= t_end) break;
        tile(e++, std::integral_constant<int, 2>{});
    }
    if (o_self != nullptr && t_mid == t_end && t_mid > t_beg)
        write_sums(o_self + static_cast<size_t>(C.start) * ncols);
    write_sums(o_all);
}

// Wide FP64 products (more than 64 columns per operator): the same eight-wave workgroups as
// k_far_wide<NSM, 1> (one operator's eight column groups, two workgroups per work item), on
// v_mfma_f64_16x16x4f64.  An FP64 left factor takes 2 KB per K-step, too large for three buffers
// of whole tiles, so every tile runs as two halves of ceil(n / 2) and n - ceil(n / 2) of its n
// K-steps (at most 11 each), in two LDS buffers of 22 KB: at the start of each half every wave
// requests its share of the next half (whole K-steps, two 1 KB buffer loads with LDS
// destination each; zeros past the half's steps) into the other buffer, and at its end waits
// for those requests, with the NH B operands it has requested since still outstanding, before
// one barrier.  A half is 11 K-steps of 64-cycle products per wave, longer than a request's
// latency.  Per wave the products are those of k_far_tiles_op<double, NSM, 1> in the same order
// (the accumulators are the FP64 sums), so both give the same sums.  Requires work items that
// do not span a chunk's own-surface boundary (plan_items, cut_self).
template <int NSM>
__global__ void __launch_bounds__(512, 2)
k_far_wide64(const Chunk* __restrict__ chunks, const FarItem* __restrict__ items,
             const int32_t* __restrict__ item_order, const int32_t* __restrict__ tile_self,
             const TileDesc* __restrict__ tiles, const double* __restrict__ tileA,
             const double* __restrict__ dens, const double* __restrict__ mom, int pad, int nwc,
             double* __restrict__ out_self, double* __restrict__ out_all,
             double* __restrict__ part) {
    constexpr int NB = NSM > DSTEPS ? NSM : DSTEPS;
    constexpr int NH = (NB + 1) / 2;    // most K-steps of a half tile
    constexpr int NREQ = (NH + 7) / 8;  // K-steps each wave requests per half
    typedef __attribute__((address_space(3))) void* lds_ptr;
    __shared__ float4 lb0[NH * 128];
    __shared__ float4 lb1[NH * 128];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wg = __builtin_amdgcn_readfirstlane(tid >> 6);  // column group of this wave
    const int c16 = lane & 15, grp = lane >> 4;
    const int ncols = 2 * pad;
    // two workgroups per work item, at b and b + 8: operator (b >> 3) & 1
    const int b = blockIdx.x;
    const int opr = (b >> 3) & 1;
    const int item = item_order[(b >> 4) * 8 + (b & 7)];
    if (item < 0) return;
    const FarItem I = items[item];
    const int chunk = I.chunk;
    const Chunk C = chunks[chunk];
    const int ntg = C.end - C.start;
    const bool mma = wg < nwc;
    const int col = opr * pad + 16 * wg + c16;
    const uint32_t boff = static_cast<uint32_t>(grp * ncols + (mma ? col : 0)) * 8u;
    const uint32_t bstep = 32u * static_cast<uint32_t>(ncols);
    v4d acc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) acc[a] = v4d{0, 0, 0, 0};
    const bool whole = I.slot < 0;
    const int t_beg = I.t0, t_end = I.t1;
    const int t_mid = whole ? t_beg + tile_self[chunk] : t_beg;
    double* const o_self = whole ? out_self : nullptr;
    double* const o_all = whole ? out_all + static_cast<size_t>(C.start) * ncols
                                : part + static_cast<size_t>(I.slot) * NT * ncols;
    auto write_sums = [&](double* out) {
        if (!mma) return;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = 16 * mt + out_row<double>(grp, q);
                if (t < ntg) out[static_cast<size_t>(t) * ncols + col] = acc[mt][q];
            }
    };
    auto b_rsrc = [&](const TileDesc& D, uint32_t rows) {
        const double* bsrc = D.kind == 0 ? mom : dens;
        return buffer_rsrc(bsrc + static_cast<size_t>(D.b_row0) * ncols,
                           rows * static_cast<uint32_t>(ncols) * 8u);
    };
    auto to_desc = [](const v4u& w) {
        const uint32_t w0 = __builtin_amdgcn_readfirstlane(w[0]);
        TileDesc D;
        D.kind = static_cast<int16_t>(w0 & 0xffffu);
        D.nstep = static_cast<int16_t>(w0 >> 16);
        D.a_blk = static_cast<int32_t>(__builtin_amdgcn_readfirstlane(w[1]));
        D.b_row0 = static_cast<int32_t>(__builtin_amdgcn_readfirstlane(w[2]));
        D.b_rows = static_cast<int32_t>(__builtin_amdgcn_readfirstlane(w[3]));
        return D;
    };
    // this wave's requests for K-steps [s0, s0 + n) of tile D's left factor (its own operator's
    // factor of a direct tile) into L: local steps wave, wave + 8, ... (the last slot may be
    // requested by more than one wave, with the same data), zeros past n
    auto request = [&](const TileDesc& D, int s0, int n, float4* L) {
        const int64_t off = D.a_off() + (D.kind == 1 ? static_cast<int64_t>(opr) * D.nstep * 256 : 0) +
                            static_cast<int64_t>(s0) * 256;
        const __amdgpu_buffer_rsrc_t ra =
            buffer_rsrc(tileA + off, n > 0 ? static_cast<uint32_t>(n) * 2048u : 0u);
#pragma unroll
        for (int k = 0; k < NREQ; ++k) {
            const int st = wg + 8 * k < NH ? wg + 8 * k : NH - 1;
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr)(L + st * 128), 16, lane * 16,
                                                     st * 2048, 0, 0);
            __builtin_amdgcn_raw_ptr_buffer_load_lds(ra, (lds_ptr)(L + st * 128 + 64), 16,
                                                     lane * 16, st * 2048 + 1024, 0, 0);
        }
    };
    // The work items of these launches never span the own-surface boundary (the plan cuts
    // every chunk there): a whole chunk's own-surface sums are its sums over all its tiles, or
    // zero when it has no own-surface tiles.
    if (o_self != nullptr && t_mid == t_beg) write_sums(o_self + static_cast<size_t>(C.start) * ncols);
    const __amdgpu_buffer_rsrc_t rt =
        buffer_rsrc(tiles + t_beg, static_cast<uint32_t>(t_end - t_beg) * 16u);
    TileDesc Te = tiles[t_beg < t_end ? t_beg : 0];
    TileDesc Tn = tiles[t_beg + 1 < t_end ? t_beg + 1 : 0];
    double bc[NH];
    {
        const int h = t_beg < t_end ? (Te.nstep + 1) / 2 : 0;
        request(Te, 0, h, lb0);
        const __amdgpu_buffer_rsrc_t rb =
            b_rsrc(Te, t_beg < t_end ? static_cast<uint32_t>(Te.b_rows) : 0u);
#pragma unroll
        for (int i = 0; i < NH; ++i) bc[i] = load_elem<double>(rb, boff, i * bstep);
    }
    __syncthreads();  // waits for every load: the first half tile is complete
    // the products of one half: n K-steps from Lc with the operands in bc, each operand register
    // then refilled with the next half's operand (step st of rbn at offset b0 + st * bstep)
    auto products = [&](const float4* Lc, int n, __amdgpu_buffer_rsrc_t rbn, uint32_t b0) {
        const int ns = mma ? n : 0;
        Quad<double> a = lds_quad<double>(Lc, 0, lane);
        uint32_t so = b0;
#pragma unroll
        for (int st = 0; st < NH; ++st) {
            Quad<double> an = a;
            if (st + 1 < NH) an = lds_quad<double>(Lc, st + 1, lane);
            if (st < ns) {
                acc[0] = Mma<double>::op(a.x, bc[st], acc[0]);
                acc[1] = Mma<double>::op(a.y, bc[st], acc[1]);
                acc[2] = Mma<double>::op(a.z, bc[st], acc[2]);
                acc[3] = Mma<double>::op(a.w, bc[st], acc[3]);
            }
            bc[st] = load_elem<double>(rbn, boff, so);
            so = next_step(so, bstep);
            a = an;
        }
    };
    // this wave's requests of the next half were made before the NH B-operand loads that
    // followed them (vmcnt field split over bits 3:0 and 15:14; expcnt and lgkmcnt not waited
    // for); the barrier then makes every wave's part visible and frees the buffer just read
    auto end_half = [&]() {
        constexpr int VM = NH;
        static_assert(VM < 64, "vmcnt range");
        __builtin_amdgcn_s_waitcnt((VM & 15) | (7 << 4) | (15 << 8) | ((VM >> 4) << 14));
        // (the empty statements keep the compiler from moving memory accesses across the
        // barrier, which itself orders none)
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };
    for (int e = t_beg; e < t_end; ++e) {
        const v4u dn = __builtin_amdgcn_raw_buffer_load_b128(
            rt, 0, static_cast<uint32_t>(e + 2 - t_beg) * 16u, 0);
        const int n = Te.nstep, h = (n + 1) / 2;
        // first half: reads lb0, requests the second half of this tile into lb1
        request(Te, h, n - h, lb1);
        products(lb0, h, b_rsrc(Te, static_cast<uint32_t>(Te.b_rows)), static_cast<uint32_t>(h) * bstep);
        end_half();
        // second half: reads lb1, requests the first half of the next tile into lb0
        const bool more = e + 1 < t_end;
        const int hn = more ? (Tn.nstep + 1) / 2 : 0;
        request(Tn, 0, hn, lb0);
        products(lb1, n - h, b_rsrc(Tn, more ? static_cast<uint32_t>(Tn.b_rows) : 0u), 0u);
        end_half();
        Te = Tn;
        Tn = to_desc(dn);
    }
    if (o_self != nullptr && t_mid == t_end && t_mid > t_beg)
        write_sums(o_self + static_cast<size_t>(C.start) * ncols);
    write_sums(o_all);
}

// Sums of the chunks cut into pieces: for each target row and column, the pieces' FP64 partial
// sums added in piece order (own-surface pieces first; their sum is the own-surface result).
__global__ void __launch_bounds__(256)
k_far_reduce(const Chunk* __restrict__ chunks, const FarRed* __restrict__ red, int n_red,
             int ncols, const double* __restrict__ part, double* __restrict__ out_self,
             double* __restrict__ out_all) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int per = NT * ncols;
    if (i >= static_cast<int64_t>(n_red) * per) return;
    const FarRed R = red[i / per];
    const int rc = static_cast<int>(i % per), t = rc / ncols;
    const Chunk C = chunks[R.chunk];
    if (t >= C.end - C.start) return;
    const size_t o = static_cast<size_t>(C.start) * ncols + rc;
    double s = 0.0;
    for (int k = R.slot0; k < R.slot1; ++k) {
        if (k == R.slot0 + R.nself && out_self != nullptr) out_self[o] = s;
        s += part[static_cast<size_t>(k) * per + rc];
    }
    if (R.nself == R.slot1 - R.slot0 && out_self != nullptr) out_self[o] = s;
    out_all[o] = s;
}

// Narrow products (one or two column groups of 16 per operator, up to 16 wavelengths) without
// LDS staging.  At these widths a left-factor value feeds the matrix cores of one wave only
// (the S = 4 / G waves of a column group split each tile's K-steps, wave k taking steps k,
// k + S, ...), so each wave streams its own operands straight from HBM into registers: per
// K-step one 16-byte (FP64: 32-byte) A operand per lane, contiguous across the wave, and one B
// value.  Each operand register is reloaded with the next tile's operand right after the
// current step has used it, so a wave keeps a tile of its own loads in flight while it
// computes, and the loop holds no barrier.
// Raw buffer loads with per-tile records read zero past a tile's factor and rows.  The step
// partition, the FP32 partial per tile, its FP64 running sum and the wave-order addition at
// the end are those of k_far_tiles_op's narrow form, so both give identical sums.
template <class T, int NSM, int S>
__global__ void __launch_bounds__(256, sizeof(T) == 4 && NSM <= 21 ? 3 : 2)
k_far_stream(const Chunk* __restrict__ chunks, const FarItem* __restrict__ items,
             const int32_t* __restrict__ item_order, const int32_t* __restrict__ tile_self,
             const TileDesc* __restrict__ tiles, const T* __restrict__ tileA,
             const T* __restrict__ dens, const T* __restrict__ mom, int pad, int nwc,
             double* __restrict__ out_self, double* __restrict__ out_all,
             double* __restrict__ part) {
    static_assert(S == 2 || S == 4, "narrow products only");
    constexpr uint32_t ES = sizeof(T);
    constexpr int G = 4 / S;                   // column groups per workgroup
    constexpr int NA = NSM > DSTEPS ? NSM : DSTEPS;
    constexpr int NBS = (NA + S - 1) / S;      // operand registers per wave
    using Acc = typename Mma<T>::acc;
    __shared__ double red[G][16][64];          // wave-order addition of the partial sums
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = lane >> 4, c16 = lane & 15;
    const int ncols = 2 * pad;
    const int b = blockIdx.x;
    const int opr = (b >> 3) & 1;              // 0: K columns, 1: V columns
    const int kpart = wave % S;                // this wave's share of the K-steps
    const int wg = wave / S;                   // column group of this wave
    const int item = item_order[(b >> 4) * 8 + (b & 7)];
    if (item < 0) return;
    const FarItem I = items[item];
    const int chunk = I.chunk;
    const Chunk C = chunks[chunk];
    const int ntg = C.end - C.start;
    const bool mma = wg < nwc;
    const int col = opr * pad + 16 * wg + c16;
    const uint32_t boff = static_cast<uint32_t>(grp * ncols + (mma ? col : 0)) * ES;
    const uint32_t bstep = 4u * ES * static_cast<uint32_t>(ncols);
    // a whole chunk, or a piece that writes its partial sums to its scratch block
    const bool whole = I.slot < 0;
    const int t_beg = I.t0, t_end = I.t1;
    const int t_mid = whole ? t_beg + tile_self[chunk] : t_beg;
    double* const o_self = whole ? out_self : nullptr;
    double* const o_all = whole ? out_all + static_cast<size_t>(C.start) * ncols
                                : part + static_cast<size_t>(I.slot) * NT * ncols;
    Acc acc[4];
    double run[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        acc[a] = Acc{0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 4; ++q) run[a][q] = 0.0;
    }
    auto own = [&](int mt, int q) -> double {
        if constexpr (sizeof(T) == 4) return run[mt][q];
        else return acc[mt][q];
    };
    auto write_sums = [&](double* out) {
        double sum[4][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int q = 0; q < 4; ++q) sum[mt][q] = own(mt, q);
        for (int k = 1; k < S; ++k) {
            if (kpart == k)
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int q = 0; q < 4; ++q) red[wg][4 * mt + q][lane] = own(mt, q);
            __syncthreads();
            if (kpart == 0)
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int q = 0; q < 4; ++q) sum[mt][q] += red[wg][4 * mt + q][lane];
            __syncthreads();
        }
        if (!mma || kpart != 0) return;
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = 16 * mt + out_row<T>(grp, q);
                if (t < ntg) out[static_cast<size_t>(t) * ncols + col] = sum[mt][q];
            }
    };
    // operand sources of tile e (empty records past the chunk's last tile)
    auto a_rsrc = [&](int e) {
        if (e >= t_end) return buffer_rsrc(tileA, 0u);
        const TileDesc D = tiles[e];
        const int64_t off = D.a_off() + (D.kind == 1 ? static_cast<int64_t>(opr) * D.nstep * 256 : 0);
        return buffer_rsrc(tileA + off, static_cast<uint32_t>(D.nstep) * 256u * ES);
    };
    auto b_rsrc = [&](int e) {
        if (e >= t_end) return buffer_rsrc(dens, 0u);
        const TileDesc D = tiles[e];
        const T* src = D.kind == 0 ? mom : dens;
        return buffer_rsrc(src + static_cast<size_t>(D.b_row0) * ncols,
                           static_cast<uint32_t>(D.b_rows) * static_cast<uint32_t>(ncols) * ES);
    };
    // this lane's A operand of K-step st: 4 consecutive elements (the four target tiles)
    auto load_a = [&](__amdgpu_buffer_rsrc_t ra, int st) {
        Quad<T> q;
        if constexpr (sizeof(T) == 4) {
            const v4u v = __builtin_amdgcn_raw_buffer_load_b128(ra, lane * 16, st * 1024, 0);
            q.x = __uint_as_float(v[0]);
            q.y = __uint_as_float(v[1]);
            q.z = __uint_as_float(v[2]);
            q.w = __uint_as_float(v[3]);
        } else {
            const v4u lo = __builtin_amdgcn_raw_buffer_load_b128(ra, lane * 16, st * 2048, 0);
            const v4u hi = __builtin_amdgcn_raw_buffer_load_b128(ra, lane * 16, st * 2048 + 1024, 0);
            q.x = __builtin_bit_cast(double, make_uint2(lo[0], lo[1]));
            q.y = __builtin_bit_cast(double, make_uint2(lo[2], lo[3]));
            q.z = __builtin_bit_cast(double, make_uint2(hi[0], hi[1]));
            q.w = __builtin_bit_cast(double, make_uint2(hi[2], hi[3]));
        }
        return q;
    };
    Quad<T> a[NBS];
    T bv[NBS];
    {
        const __amdgpu_buffer_rsrc_t ra = a_rsrc(t_beg), rb = b_rsrc(t_beg);
#pragma unroll
        for (int i = 0; i < NBS; ++i) {
            a[i] = load_a(ra, kpart + S * i);
            bv[i] = load_elem<T>(rb, boff, (kpart + S * i) * bstep);
        }
    }
    auto tile = [&](int e) {
        const __amdgpu_buffer_rsrc_t ran = a_rsrc(e + 1), rbn = b_rsrc(e + 1);
#pragma unroll
        for (int i = 0; i < NBS; ++i) {
            const int st = kpart + S * i;
            if (st < NA && mma) {  // past a tile's own steps the operands read zero
                acc[0] = Mma<T>::op(a[i].x, bv[i], acc[0]);
                acc[1] = Mma<T>::op(a[i].y, bv[i], acc[1]);
                acc[2] = Mma<T>::op(a[i].z, bv[i], acc[2]);
                acc[3] = Mma<T>::op(a[i].w, bv[i], acc[3]);
            }
            a[i] = load_a(ran, st);
            bv[i] = load_elem<T>(rbn, boff, st * bstep);
            // FP32: this wave's partial of every DSTEPS K-steps of the tile joins the FP64
            // running sums (the staged kernel's schedule)
            if constexpr (sizeof(T) == 4) {
                if ((i + 1) % (DSTEPS / S) == 0 || i + 1 == NBS) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) run[q][r] += static_cast<double>(acc[q][r]);
                        acc[q] = Acc{0, 0, 0, 0};
                    }
                }
            }
        }
    };
    for (int e = t_beg; e < t_mid; ++e) tile(e);
    if (o_self != nullptr) write_sums(o_self + static_cast<size_t>(C.start) * ncols);
    for (int e = t_mid; e < t_end; ++e) tile(e);
    write_sums(o_all);
}

// ------------------------------------------------------------------------------- P2M, MFMA
// The folded moments of an expanded box are linear in the densities of its panels with
// geometry-only weights: M[term][col] = sum_j A[term][j] dens[j][col], A[term][j] the folded
// node polynomial of panel j (V polynomial for the V columns, K polynomial for the K columns).
// k_build_p2m_tiles stores A once per geometry, segment by segment (P2MSeg: at most 128 panels
// of one box), as [step][row tile][lane] with step = 4 panels and lane l holding
// A[16 rt + l % 16][4 step + l / 16] (the operand order of v_mfma_f32_16x16x4f32 and of
// v_mfma_f64_16x16x4f64); the K block of a segment follows its V block.  One pass writes the
// FP32 and / or FP64 copies (null when not kept), from the FP64 panel records when the geometry
// has them.  k_p2m_mfma then forms each segment's moments on matrix cores, in the precision of
// the product.
template <int P>
constexpr int p2m_row_tiles() { return (Expansion<P>::NR + 15) / 16; }

// Index of term (x, y, z) in the full list (by degree, then x and y descending).
__device__ __forceinline__ int full_term(int x, int y, int z) {
    const int n = x + y + z, a = n - x;
    return n * (n + 1) * (n + 2) / 6 + a * (a + 1) / 2 + (a - y);
}

// One block per segment, PB panels at a time with TPP threads each: the node polynomials of a
// panel go to LDS (each thread a share of the terms, nodes summed in order), the kz >= 2 terms
// are folded level by level (each destination gathers its two sources in the order of the
// sequential fold), and the folded terms are stored.
template <class S, int P>
__global__ void __launch_bounds__(128)
k_build_p2m_tiles(const Box* __restrict__ boxes, const P2MSeg* __restrict__ segs,
                  const int64_t* __restrict__ aoff, const double* __restrict__ cen,
                  const S* __restrict__ src, int K, float* __restrict__ A32,
                  double* __restrict__ A64) {
    using E = Expansion<P>;
    constexpr E ex{};
    constexpr int NF = E::NF, NR = E::NR, RT = p2m_row_tiles<P>();
    constexpr int PB = P <= 10 ? 8 : 4, TPP = 128 / PB;  // LDS at most 65 KB up to P = 15
    __shared__ double poly[PB][2][NF];  // V then K polynomial of each panel of the batch
    // powers d^0..d^P of each node's offset from the box centre, per axis (at most 8 nodes)
    __shared__ double pw[PB][8][3][P + 1];
    const P2MSeg sg = segs[blockIdx.x];
    const Box B = boxes[sg.box];
    const int lp = threadIdx.x / TPP, lt = threadIdx.x % TPP;
    const int rs = 4 + 4 * K;
    const int steps = (sg.end - sg.start + 3) / 4;
    const size_t a0 = aoff[blockIdx.x], kb = static_cast<size_t>(steps) * RT * 64;
    double* pv = poly[lp][0];
    double* pk = poly[lp][1];
    for (int base = sg.start; base < sg.end; base += PB) {
        const int j = base + lp;
        const bool live = j < sg.end;
        const S* r = src + static_cast<size_t>(live ? j : sg.start) * rs;
        if (live) {
            // powers of each node's offset by successive products from 1, once per node and axis
            const double cc[3] = {cen[3 * j] - B.cx, cen[3 * j + 1] - B.cy, cen[3 * j + 2] - B.cz};
            for (int u = lt; u < 3 * K; u += TPP) {
                const int gq = u / 3, ax = u % 3;
                const double d = cc[ax] + r[4 + 4 * gq + ax];
                double* pp = pw[lp][gq][ax];
                double X = 1.0;
                pp[0] = X;
                for (int q = 1; q <= P; ++q) {
                    X *= d;
                    pp[q] = X;
                }
            }
        }
        __syncthreads();
        if (live) {
            for (int t = lt; t < NF; t += TPP) {
                const int kx = ex.fx[t], ky = ex.fy[t], kz = ex.fz[t];
                double v = 0.0, k = 0.0;
                for (int gq = 0; gq < K; ++gq) {
                    const double* px = pw[lp][gq][0];
                    const double* py = pw[lp][gq][1];
                    const double* pz = pw[lp][gq][2];
                    const double w = r[7 + 4 * gq];
                    const double X = px[kx], Y = py[ky], Z = pz[kz];
                    v += w * X * Y * Z;
                    double gs = 0.0;
                    if (kx > 0) gs += r[0] * kx * px[kx - 1] * Y * Z;
                    if (ky > 0) gs += r[1] * ky * X * py[ky - 1] * Z;
                    if (kz > 0) gs += r[2] * kz * X * Y * pz[kz - 1];
                    k += w * gs;
                }
                pv[t] = v;
                pk[t] = k;
            }
        }
        __syncthreads();
        // fold: level z feeds level z - 2, whose term (x, y) receives c_y M(x, y - 2, z) and
        // then c_x M(x - 2, y, z), c = -(k - 1) k / ((z - 1) z)
        for (int z = P; z >= 2; --z) {
            const int L = P - z + 2;  // x + y <= L at level z - 2
            const double den = double(z - 1) * double(z);
            for (int u = lt; u < (L + 1) * (L + 2) / 2; u += TPP) {
                int x = 0, rem = u;
                while (rem > L - x) {
                    rem -= L - x + 1;
                    ++x;
                }
                const int y = rem;
                if (!live) continue;
                const int dst = full_term(x, y, z - 2);
                double v = pv[dst], k = pk[dst];
                if (y >= 2) {
                    const double c = -double(y - 1) * double(y) / den;
                    const int sidx = full_term(x, y - 2, z);
                    v += c * pv[sidx];
                    k += c * pk[sidx];
                }
                if (x >= 2) {
                    const double c = -double(x - 1) * double(x) / den;
                    const int sidx = full_term(x - 2, y, z);
                    v += c * pv[sidx];
                    k += c * pk[sidx];
                }
                pv[dst] = v;
                pk[dst] = k;
            }
            __syncthreads();
        }
        if (live) {
            const int p = j - sg.start, st = p >> 2, kk = p & 3;
            for (int q = lt; q < NR; q += TPP) {
                const int rt = q >> 4, lane = (q & 15) + 16 * kk;
                const size_t idx = a0 + (static_cast<size_t>(st) * RT + rt) * 64 + lane;
                const double v = pv[ex.rfull[q]], k = pk[ex.rfull[q]];
                if (A32 != nullptr) {
                    A32[idx] = static_cast<float>(v);
                    A32[idx + kb] = static_cast<float>(k);
                }
                if (A64 != nullptr) {
                    A64[idx] = v;
                    A64[idx + kb] = k;
                }
            }
        }
        __syncthreads();
    }
}

// Workgroup = (segment, operator, column half): 4 waves, each 16 columns of one operator.
template <class T, int RT, int NR>
__global__ void __launch_bounds__(256)
k_p2m_mfma(const P2MSeg* __restrict__ segs, const int64_t* __restrict__ aoff,
           const T* __restrict__ A, const T* __restrict__ dens, int pad, int nwc,
           T* __restrict__ mom, T* __restrict__ part) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c16 = lane & 15, grp = lane >> 4;
    const int opr = blockIdx.y & 1, wg = wave + 4 * (blockIdx.y >> 1);
    if (wg >= nwc) return;
    const int ncols = 2 * pad;
    const int col = opr * pad + 16 * wg + c16;
    const P2MSeg sg = segs[blockIdx.x];
    const int np = sg.end - sg.start, steps = (np + 3) / 4;
    const T* Ab = A + aoff[blockIdx.x] + (opr == 0 ? static_cast<size_t>(steps) * RT * 64 : 0);
    const T* Db = dens + static_cast<size_t>(sg.start) * ncols + col;
    typename Mma<T>::acc acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t] = typename Mma<T>::acc{0, 0, 0, 0};
#pragma unroll 2
    for (int st = 0; st < steps; ++st) {
        const int p = 4 * st + grp;
        const T b = Db[static_cast<size_t>(p < np ? p : 0) * ncols];
        const T bb = p < np ? b : T(0);
        const T* a = Ab + static_cast<size_t>(st) * RT * 64 + lane;
#pragma unroll
        for (int t = 0; t < RT; ++t) acc[t] = Mma<T>::op(a[t * 64], bb, acc[t]);
    }
    T* out = sg.slot < 0 ? mom + static_cast<size_t>(sg.mslot) * NR * ncols
                         : part + static_cast<size_t>(sg.slot) * NR * ncols;
#pragma unroll
    for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int q = 16 * t + out_row<T>(grp, i);
            if (q < NR) out[static_cast<size_t>(q) * ncols + col] = acc[t][i];
        }
}

// ---- geometry-only tiles of the far-field products (built once per geometry)
// Expansion tile of list entry e: Taylor coefficients of the chunk's 64 targets for its box.
// tileA32 (FP64 builds, may be null): the same values rounded to FP32, at the same offsets.
template <class T, int P>
__global__ void k_build_m2p_tiles(const Chunk* __restrict__ chunks, const Box* __restrict__ boxes,
                                  const TileDesc* __restrict__ tiles,
                                  const int32_t* __restrict__ m2p_tile,
                                  const int32_t* __restrict__ m2p_chunk,
                                  const int32_t* __restrict__ m2p_box, int n,
                                  const double* __restrict__ cen, T* __restrict__ tileA,
                                  float* __restrict__ tileA32) {
    using E = Expansion<P>;
    constexpr int NR = E::NR;
    const int e = blockIdx.x;
    if (e >= n) return;
    const int t = threadIdx.x;  // target within the chunk
    const Chunk C = chunks[m2p_chunk[e]];
    const Box B = boxes[m2p_box[e]];
    const TileDesc TD = tiles[m2p_tile[e]];
    T* A = tileA + TD.a_off();
    const int i = C.start + t;
    T F[NR];
    if (i < C.end) {
        taylor_coefficients<T, P>(static_cast<T>(B.cx - cen[3 * i]),
                                  static_cast<T>(B.cy - cen[3 * i + 1]),
                                  static_cast<T>(B.cz - cen[3 * i + 2]), F);
    } else {
#pragma unroll
        for (int q = 0; q < NR; ++q) F[q] = T(0);
    }
    const int mt = t >> 4, r16 = t & 15;
    // slice k holds terms [4 SST k, 4 SST (k + 1)) as SST K-steps, its tile right after slice
    // k - 1's in the store (zero past the last term)
    constexpr int SST = expansion_slice_steps(NR), PER = 4 * SST;
    constexpr int TOT = expansion_slices(NR) * PER;
#pragma unroll
    for (int q = 0; q < TOT; ++q) {
        const int k = q / PER, st = (q % PER) >> 2, g = q & 3;
        const size_t base = static_cast<size_t>(k) * SST * 256;
        const T v = q < NR ? F[q] : T(0);
        A[base + tile_index<T>(st, 16 * g + r16, mt)] = v;
        if (tileA32 != nullptr)
            tileA32[TD.a_off() + base + tile_index<float>(st, 16 * g + r16, mt)] = static_cast<float>(v);
    }
}


// Direct tile: far-rule single- and double-layer kernel values of the chunk's 64 targets for
// up to 4 direct_steps() consecutive source panels (zero for the target's own panel and past the
// range).  The tile's source records and centroids are staged in LDS by one contiguous copy;
// each thread keeps its target's centroid (thread t of every wave: target t).
constexpr int P2P_MAXP = 4 * 31;    // panels of a direct tile: direct_steps() <= 31
constexpr int P2P_MAXR = 4 + 4 * 8;  // record length for up to 8 far-rule nodes
template <class T>
__global__ void __launch_bounds__(256)
k_build_p2p_tiles(const Chunk* __restrict__ chunks, const TileDesc* __restrict__ tiles,
                  const int32_t* __restrict__ p2p_tile, const int32_t* __restrict__ p2p_chunk,
                  int n, const double* __restrict__ cen, const T* __restrict__ src, int K,
                  T* __restrict__ tileA, float* __restrict__ tileA32) {
    __shared__ T rec[P2P_MAXP * P2P_MAXR];
    __shared__ double cj[P2P_MAXP * 3];
    const int e = blockIdx.x;
    if (e >= n) return;
    const TileDesc TD = tiles[p2p_tile[e]];
    const Chunk C = chunks[p2p_chunk[e]];
    T* AK = tileA + TD.a_off();
    T* AV = AK + static_cast<size_t>(TD.nstep) * 256;
    float* BK = tileA32 != nullptr ? tileA32 + TD.a_off() : nullptr;
    const int rs = 4 + 4 * K, np = TD.b_rows;
    const T* rsrc = src + static_cast<size_t>(TD.b_row0) * rs;
    for (int u = threadIdx.x; u < np * rs; u += blockDim.x) rec[u] = rsrc[u];
    for (int u = threadIdx.x; u < np * 3; u += blockDim.x) cj[u] = cen[3 * static_cast<size_t>(TD.b_row0) + u];
    const int t = threadIdx.x & 63, i = C.start + t;  // every pr below has pr & 63 == t
    const bool tin = i < C.end;
    const double xi = tin ? cen[3 * i] : 0.0, yi = tin ? cen[3 * i + 1] : 0.0,
                 zi = tin ? cen[3 * i + 2] : 0.0;
    __syncthreads();
    for (int pr = threadIdx.x; pr < 64 * 4 * TD.nstep; pr += blockDim.x) {
        const int p = pr >> 6;  // panel within the tile
        const int j = TD.b_row0 + p;
        T kv = 0, kk = 0;
        if (tin && p < np && j != i) {
            const T* r = rec + p * rs;
            const T dx = static_cast<T>(xi - cj[3 * p]);
            const T dy = static_cast<T>(yi - cj[3 * p + 1]);
            const T dz = static_cast<T>(zi - cj[3 * p + 2]);
            const T sh = r[0] * dx + r[1] * dy + r[2] * dz;
            T sv = 0, sk = 0;
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
            kk = sh * sk;
        }
        const int st = p >> 2, g = p & 3, mt = t >> 4, r16 = t & 15;
        const size_t idx = tile_index<T>(st, 16 * g + r16, mt);
        AK[idx] = kk;
        AV[idx] = kv;
        if (BK != nullptr) {
            const size_t i32 = tile_index<float>(st, 16 * g + r16, mt);
            BK[i32] = static_cast<float>(kk);
            BK[static_cast<size_t>(TD.nstep) * 256 + i32] = static_cast<float>(kv);
        }
    }
}

// Near-singular pairs and the singular self-term folded into the direct tiles: the far-rule
// value of a near pair (i, j) plus its fine-minus-far correction is its fine-rule value
// (section "Integral evaluation"), and V_ii joins the otherwise empty self pair.  Every near
// pair lies in a direct tile of its target's chunk (a box is never expanded for targets that
// could be near-singular to it), so the tiles then carry the whole operator.  Thread = one
// near-singular entry (e < nnz) or one self pair (e = nnz + i): every thread adds to its own
// tile entry once, so no two threads touch one entry; pairs without a tile are counted (the
// caller then rebuilds the tiles without folding).
template <class T>
__global__ void k_fold_near(const Chunk* __restrict__ chunks, int n_chunks,
                            const int32_t* __restrict__ dt_off, const int32_t* __restrict__ dt_row0,
                            const int32_t* __restrict__ dt_tile,
                            const TileDesc* __restrict__ tiles, const int64_t* __restrict__ off,
                            const int32_t* __restrict__ col, const double* __restrict__ dv,
                            const double* __restrict__ dk, const double* __restrict__ vself,
                            int N, int64_t nnz, T* __restrict__ tileA,
                            float* __restrict__ tileA32, int32_t* __restrict__ missing) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nnz + N) return;
    int i, j;
    double add_k, add_v;
    if (e < nnz) {
        // the row of entry e: the last target whose first entry is at or before e (an empty
        // row shares its offset with the next one)
        int a = 0, b = N - 1;
        while (a < b) {
            const int mid = (a + b + 1) / 2;
            if (off[mid] <= e) a = mid;
            else b = mid - 1;
        }
        i = a;
        j = col[e];
        add_k = dk[e];
        add_v = dv[e];
    } else {
        i = static_cast<int>(e - nnz);
        j = i;
        add_k = 0.0;
        add_v = vself[i];
    }
    int lo = 0, hi = n_chunks - 1;  // the chunk holding target i (chunks are in target order)
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (chunks[mid].start <= i) lo = mid;
        else hi = mid - 1;
    }
    const int t = i - chunks[lo].start;
    const int d0 = dt_off[lo], d1 = dt_off[lo + 1];
    // the chunk's direct tiles sorted by first source panel: the last one starting at or
    // before j holds j if j is inside its range
    auto place = [&](int j, double add_k, double add_v) {
        int a = d0, b = d1 - 1;
        if (b < a || dt_row0[a] > j) return false;
        while (a < b) {
            const int mid = (a + b + 1) / 2;
            if (dt_row0[mid] <= j) a = mid;
            else b = mid - 1;
        }
        const TileDesc TD = tiles[dt_tile[a]];
        const int p = j - TD.b_row0;
        if (p >= TD.b_rows) return false;
        T* AK = tileA + TD.a_off();
        T* AV = AK + static_cast<size_t>(TD.nstep) * 256;
        const int st = p >> 2, gq = p & 3, mt = t >> 4, r16 = t & 15;
        const size_t idx = tile_index<T>(st, 16 * gq + r16, mt);
        AK[idx] = static_cast<T>(static_cast<double>(AK[idx]) + add_k);
        AV[idx] = static_cast<T>(static_cast<double>(AV[idx]) + add_v);
        if (tileA32 != nullptr) {  // FP32 copy of FP64 tiles: the folded values, rounded
            float* BK = tileA32 + TD.a_off();
            const size_t i32 = tile_index<float>(st, 16 * gq + r16, mt);
            BK[i32] = static_cast<float>(AK[idx]);
            BK[static_cast<size_t>(TD.nstep) * 256 + i32] = static_cast<float>(AV[idx]);
        }
        return true;
    };
    if (!place(j, add_k, add_v)) atomicAdd(missing, 1);
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

template <class T>
const T* src_of(const Geometry& g);
template <>
const float* src_of<float>(const Geometry& g) { return g.src32.p; }
template <>
const double* src_of<double>(const Geometry& g) { return g.src64.p; }

template <class T, int P, int CPT>
void launch_far_p(Geometry& g, int pad, const T* dens, const T* mom, double* os, double* oa,
                  hipStream_t s) {
    const int threads = NT * (pad / CPT);
    hipLaunchKernelGGL((k_far<T, P, CPT>), dim3(g.n_chunks), dim3(threads), 0, s, g.chunks.p,
                       g.boxes.p, g.m2p_off.p, g.m2p_box.p, g.m2p_self.p, g.p2p_off.p,
                       g.p2p_rng.p, g.p2p_self.p, g.cen.p, src_of<T>(g), g.K, dens, mom,
                       g.mom_slot.p, pad, os, oa);
    LSPR_HIP(hipGetLastError());
}

template <class T, int P>
void launch_p2m_p(Geometry& g, int pad, const T* dens, T* mom, hipStream_t s) {
    if (g.n_seg == 0) return;
    const int ncols = 2 * pad;
    const int nr = Expansion<P>::NR;
    T* part = nullptr;
    if (g.n_slots > 0) {
        part = reinterpret_cast<T*>(
            workspace(g, g.ws_part, static_cast<size_t>(g.n_slots) * nr * ncols * sizeof(T)));
    }
    const dim3 grid(g.n_seg, (ncols + P2M_THREADS - 1) / P2M_THREADS);
    hipLaunchKernelGGL((k_p2m<T, P>), grid, dim3(P2M_THREADS), 0, s, g.boxes.p, g.p2m_seg.p,
                       g.cen.p, src_of<T>(g), g.K, dens, pad, mom, part);
    LSPR_HIP(hipGetLastError());
    if (g.n_red > 0) {
        const int64_t tot = static_cast<int64_t>(g.n_red) * nr * ncols;
        hipLaunchKernelGGL(k_p2m_reduce<T>, dim3((tot + 255) / 256), dim3(256), 0, s,
                           g.p2m_red.p, g.n_red, nr, ncols, part, mom);
        LSPR_HIP(hipGetLastError());
    }
}

template <class T>
const T* tiles_of(const Geometry& g);
template <>
const float* tiles_of<float>(const Geometry& g) { return g.tileA.p; }
template <>
const double* tiles_of<double>(const Geometry& g) { return g.tileA64.p; }

// Work items of a launch of pad columns per operator: plan 0 up to 16 wavelengths, 1 up to 32,
// 2 above.
inline const Geometry::FarPlan& far_plan_for(const Geometry& g, int pad) {
    return g.far_plan[pad > 64 ? 2 : (pad > 32 ? 1 : 0)];
}

}  // namespace

// Scratch bytes of the pieces' partial sums of a launch of pad columns per operator.
size_t far_part_bytes(const Geometry& g, int pad) {
    return static_cast<size_t>(far_plan_for(g, pad).n_slots) * NT * 2 * pad * sizeof(double);
}

namespace {

// Sums of the chunks a launch cut into pieces (after the far-field kernel, same stream).
void launch_far_reduce(Geometry& g, const Geometry::FarPlan& fp, int pad, const double* part,
                       double* os, double* oa, hipStream_t s) {
    if (fp.n_red == 0) return;
    const int64_t tot = static_cast<int64_t>(fp.n_red) * NT * 2 * pad;
    hipLaunchKernelGGL(k_far_reduce, dim3((tot + 255) / 256), dim3(256), 0, s, g.chunks.p,
                       fp.red.p, fp.n_red, 2 * pad, part, os, oa);
    LSPR_HIP(hipGetLastError());
}

template <class T, int NSM, int S, int OPS = 1>
void launch_far_tiles_op_s(Geometry& g, int pad, int abuf, const T* dens, const T* mom,
                           double* os, double* oa, hipStream_t s) {
    const int halves = pad > 64 ? 2 : 1;
    const Geometry::FarPlan& fp = far_plan_for(g, pad);
    double* part = nullptr;
    if (fp.n_slots > 0)
        part = reinterpret_cast<double*>(workspace(g, g.ws_fpart, far_part_bytes(g, pad)));
    const int nblk = fp.n_order * (OPS == 2 ? 1 : 2) * halves;
    // the left factor (OPS = 2: a direct tile's two), then (S > 1) one slot of FP64 sums per
    // column group for the final additions
    const size_t ab = OPS == 2 ? 2 * static_cast<size_t>(abuf) : abuf;
    const size_t lds = ab * sizeof(T) + (S > 1 ? OPS * (4 / S) * 16 * 64 * 8 : 0);
    if (lds > 64 * 1024)
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_far_tiles_op<T, NSM, S, OPS>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                  static_cast<int>(lds));
    hipLaunchKernelGGL((k_far_tiles_op<T, NSM, S, OPS>), dim3(nblk), dim3(256 * OPS), lds, s,
                       g.chunks.p, fp.items.p, fp.order.p, g.tile_self.p, g.tiles.p,
                       tiles_of<T>(g), dens, mom, pad, pad / 16, halves, os, oa, part);
    LSPR_HIP(hipGetLastError());
    launch_far_reduce(g, fp, pad, part, os, oa, s);
}

template <class T, int NSM, int S>
void launch_far_stream(Geometry& g, int pad, const T* dens, const T* mom, double* os,
                       double* oa, hipStream_t s) {
    const Geometry::FarPlan& fp = far_plan_for(g, pad);
    double* part = nullptr;
    if (fp.n_slots > 0)
        part = reinterpret_cast<double*>(workspace(g, g.ws_fpart, far_part_bytes(g, pad)));
    const int nblk = fp.n_order * 2;
    hipLaunchKernelGGL((k_far_stream<T, NSM, S>), dim3(nblk), dim3(256), 0, s, g.chunks.p,
                       fp.items.p, fp.order.p, g.tile_self.p, g.tiles.p, tiles_of<T>(g), dens,
                       mom, pad, pad / 16, os, oa, part);
    LSPR_HIP(hipGetLastError());
    launch_far_reduce(g, fp, pad, part, os, oa, s);
}

template <int NSM, int S>
void launch_far_wide(Geometry& g, int pad, const float* dens, const float* mom, double* os,
                     double* oa, hipStream_t s) {
    const Geometry::FarPlan& fp = far_plan_for(g, pad);
    double* part = nullptr;
    if (fp.n_slots > 0)
        part = reinterpret_cast<double*>(workspace(g, g.ws_fpart, far_part_bytes(g, pad)));
    const int nblk = fp.n_order * 2;
    hipLaunchKernelGGL((k_far_wide<NSM, S>), dim3(nblk), dim3(512), 0, s, g.chunks.p, fp.items.p,
                       fp.order.p, g.tile_self.p, g.tiles.p, g.tileA.p, dens, mom, pad, pad / 16,
                       os, oa, part);
    LSPR_HIP(hipGetLastError());
    launch_far_reduce(g, fp, pad, part, os, oa, s);
}

template <int NSM>
void launch_far_wide64(Geometry& g, int pad, const double* dens, const double* mom, double* os,
                       double* oa, hipStream_t s) {
    const Geometry::FarPlan& fp = far_plan_for(g, pad);
    double* part = nullptr;
    if (fp.n_slots > 0)
        part = reinterpret_cast<double*>(workspace(g, g.ws_fpart, far_part_bytes(g, pad)));
    const int nblk = fp.n_order * 2;
    hipLaunchKernelGGL((k_far_wide64<NSM>), dim3(nblk), dim3(512), 0, s, g.chunks.p, fp.items.p,
                       fp.order.p, g.tile_self.p, g.tiles.p, g.tileA64.p, dens, mom, pad,
                       pad / 16, os, oa, part);
    LSPR_HIP(hipGetLastError());
    launch_far_reduce(g, fp, pad, part, os, oa, s);
}

// one column group per operator: four waves share it; two: two waves each; more: one each.
// Narrow products stage their left factors in LDS, or stream their operands (k_far_stream)
// when the geometry asks for it.
template <class T, int NSM>
void launch_far_tiles_op(Geometry& g, int pad, int abuf, const T* dens, const T* mom,
                         double* os, double* oa, hipStream_t s) {
    const int groups = pad / 16;
    // FP32 products of up to 32 columns per operator at P = 8 or 15: eight-wave workgroups that
    // read the left factors straight into LDS, with 4 or 8 waves per column group (two waves
    // per group, for three or four groups, need more than four waves' registers per SIMD)
    if constexpr (std::is_same<T, float>::value && (NSM == 21 || NSM == 16)) {
        if (!g.four_wave && !g.stream_narrow && !g.pair_narrow && groups <= 2) {
            if (groups == 1) launch_far_wide<NSM, 8>(g, pad, dens, mom, os, oa, s);
            else launch_far_wide<NSM, 4>(g, pad, dens, mom, os, oa, s);
            return;
        }
    }
    if (groups == 1) {
        if (g.stream_narrow) launch_far_stream<T, NSM, 4>(g, pad, dens, mom, os, oa, s);
        else if (g.pair_narrow) launch_far_tiles_op_s<T, NSM, 4, 2>(g, pad, abuf, dens, mom, os, oa, s);
        else launch_far_tiles_op_s<T, NSM, 4>(g, pad, abuf, dens, mom, os, oa, s);
    } else if (groups == 2) {
        if (g.stream_narrow) launch_far_stream<T, NSM, 2>(g, pad, dens, mom, os, oa, s);
        else if (g.pair_narrow) launch_far_tiles_op_s<T, NSM, 2, 2>(g, pad, abuf, dens, mom, os, oa, s);
        else launch_far_tiles_op_s<T, NSM, 2>(g, pad, abuf, dens, mom, os, oa, s);
    } else if (g.pair_ops) {
        launch_far_tiles_op_s<T, NSM, 1, 2>(g, pad, abuf, dens, mom, os, oa, s);
    } else {
        if constexpr (std::is_same<T, float>::value && NSM <= 21) {
            // FP32 above 64 columns per operator: both column halves in one workgroup (up to
            // P = 8: at longer slices its registers exceed four waves per SIMD)
            if (groups > 4 && !g.four_wave) {
                launch_far_wide<NSM, 1>(g, pad, dens, mom, os, oa, s);
                return;
            }
        }
        if constexpr (std::is_same<T, double>::value && NSM <= 21) {
            // FP64 above 64 columns per operator: the same, in half tiles
            if (groups > 4 && !g.four_wave) {
                launch_far_wide64<NSM>(g, pad, dens, mom, os, oa, s);
                return;
            }
        }
        launch_far_tiles_op_s<T, NSM, 1>(g, pad, abuf, dens, mom, os, oa, s);
    }
}

template <class T>
void launch_far_tiles(Geometry& g, int pad, const T* dens, const T* mom, double* os,
                      double* oa, hipStream_t s) {
    const int nsm = expansion_slice_steps(g.n_terms);
    const int abuf = direct_steps(g.n_terms) * 256;  // largest part a workgroup stages
#define LSPR_FAR_OP(NSM_)                                                                    \
    case NSM_:                                                                               \
        launch_far_tiles_op<T, NSM_>(g, pad, abuf, dens, mom, os, oa, s);                    \
        return;
    switch (nsm) {  // K-steps of an expansion slice for P = 2, 4, 6, 12, 15, 8, 10
        LSPR_FAR_OP(3)
        LSPR_FAR_OP(7)
        LSPR_FAR_OP(13)
        LSPR_FAR_OP(15)
        LSPR_FAR_OP(16)
        LSPR_FAR_OP(21)
        LSPR_FAR_OP(31)
        default: throw Error(LSPR_E_INVALID, "unsupported expansion order");
    }
#undef LSPR_FAR_OP
}

inline const float* p2m_tiles_of(const Geometry& g, const float*) { return g.p2mA.p; }
inline const double* p2m_tiles_of(const Geometry& g, const double*) { return g.p2mA64.p; }

template <class T, int P>
void launch_p2m_mfma(Geometry& g, int pad, const T* dens, T* mom, hipStream_t s) {
    if (g.n_seg == 0) return;
    constexpr int NR = Expansion<P>::NR, RT = p2m_row_tiles<P>();
    const int ncols = 2 * pad;
    T* part = nullptr;
    if (g.n_slots > 0) {
        part = reinterpret_cast<T*>(
            workspace(g, g.ws_part, static_cast<size_t>(g.n_slots) * NR * ncols * sizeof(T)));
    }
    const int halves = pad > 64 ? 2 : 1;
    hipLaunchKernelGGL((k_p2m_mfma<T, RT, NR>), dim3(g.n_seg, 2 * halves), dim3(256), 0, s,
                       g.p2m_seg.p, g.p2m_aoff.p, p2m_tiles_of(g, dens), dens, pad, pad / 16,
                       mom, part);
    LSPR_HIP(hipGetLastError());
    if (g.n_red > 0) {
        const int64_t tot = static_cast<int64_t>(g.n_red) * NR * ncols;
        hipLaunchKernelGGL(k_p2m_reduce<T>, dim3((tot + 255) / 256), dim3(256), 0, s,
                           g.p2m_red.p, g.n_red, NR, ncols, part, mom);
        LSPR_HIP(hipGetLastError());
    }
}

// Moments on matrix cores when the geometry holds polynomial tiles of the product's
// precision; false otherwise.
template <class T>
bool launch_p2m_tiles(Geometry& g, const Cols& c, const T* dens, T* mom, hipStream_t s) {
    if (!c.mfma || p2m_tiles_of(g, dens) == nullptr) return false;
    switch (g.P) {
        case 2: launch_p2m_mfma<T, 2>(g, c.pad, dens, mom, s); break;
        case 4: launch_p2m_mfma<T, 4>(g, c.pad, dens, mom, s); break;
        case 6: launch_p2m_mfma<T, 6>(g, c.pad, dens, mom, s); break;
        case 8: launch_p2m_mfma<T, 8>(g, c.pad, dens, mom, s); break;
        case 10: launch_p2m_mfma<T, 10>(g, c.pad, dens, mom, s); break;
        case 12: launch_p2m_mfma<T, 12>(g, c.pad, dens, mom, s); break;
        case 15: launch_p2m_mfma<T, 15>(g, c.pad, dens, mom, s); break;
        default: throw Error(LSPR_E_INVALID, "expansion order must be 2, 4, 6, 8, 10, 12 or 15");
    }
    return true;
}

// Allocations and the offset table in the order of s; the fills and the builder on s2, after
// that point of s (the caller waits for s2).
template <int P>
void build_p2m_tiles_p(Geometry& g, hipStream_t s, hipStream_t s2) {
    constexpr int RT = p2m_row_tiles<P>();
    const std::vector<P2MSeg>& segs = g.p2m_seg_h;
    LSPR_REQUIRE(static_cast<int>(segs.size()) == g.n_seg, LSPR_E_INVALID,
                 "moment segments missing on the host");
    std::vector<int64_t> off(g.n_seg);
    int64_t tot = 0;
    for (int k = 0; k < g.n_seg; ++k) {
        off[k] = tot;
        tot += 2ll * ((segs[k].end - segs[k].start + 3) / 4) * RT * 64;
    }
    g.p2m_aoff.alloc(g.n_seg);
    copy_sync(g.p2m_aoff.p, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice, s);
    if (g.tileA.p != nullptr) g.p2mA.alloc(std::max<int64_t>(tot, 1));
    if (g.tileA64.p != nullptr) g.p2mA64.alloc(std::max<int64_t>(tot, 1));
    hipEvent_t ev = nullptr;
    LSPR_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    const hipError_t e1 = hipEventRecord(ev, s);
    const hipError_t e2 = e1 == hipSuccess ? hipStreamWaitEvent(s2, ev, 0) : e1;
    (void)hipEventDestroy(ev);
    LSPR_HIP(e2);
    if (g.p2mA.p != nullptr) LSPR_HIP(hipMemsetAsync(g.p2mA.p, 0, g.p2mA.bytes(), s2));
    if (g.p2mA64.p != nullptr) LSPR_HIP(hipMemsetAsync(g.p2mA64.p, 0, g.p2mA64.bytes(), s2));
    if (g.src64.p != nullptr)
        hipLaunchKernelGGL((k_build_p2m_tiles<double, P>), dim3(g.n_seg), dim3(128), 0, s2,
                           g.boxes.p, g.p2m_seg.p, g.p2m_aoff.p, g.cen.p, g.src64.p, g.K,
                           g.p2mA.p, g.p2mA64.p);
    else
        hipLaunchKernelGGL((k_build_p2m_tiles<float, P>), dim3(g.n_seg), dim3(128), 0, s2,
                           g.boxes.p, g.p2m_seg.p, g.p2m_aoff.p, g.cen.p, g.src32.p, g.K,
                           g.p2mA.p, g.p2mA64.p);
    LSPR_HIP(hipGetLastError());
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
        default: throw Error(LSPR_E_INVALID, "expansion orders above 10 run only from matrix-core tiles");
    }
}

template <class T>
void apply_far_t(Geometry& g, const Cols& c, const T* dens, double* os, double* oa,
                 hipStream_t s) {
    LSPR_REQUIRE(src_of<T>(g) != nullptr, LSPR_E_INVALID,
                 "the geometry was not built for products in this precision");
    const double nc = c.ncol;                     // used real columns per operator
    const double esz = sizeof(T);
    const double dens_bytes = double(g.N) * 2 * c.pad * esz;
    const double out_bytes = double(g.N) * 2 * c.pad * 8 * (os ? 2 : 1);
    const int NF = (g.P + 1) * (g.P + 2) * (g.P + 3) / 6;
    const double mom_bytes = double(g.mom_boxes.size()) * g.n_terms * 2 * c.pad * esz;
    const bool fp64 = sizeof(T) == 8;
    T* mom = nullptr;
    if (!g.mom_boxes.empty()) {
        const size_t need = g.mom_boxes.size() * g.n_terms * 2 * c.pad * sizeof(T);
        mom = reinterpret_cast<T*>(workspace(g, g.ws_mom, need));
        // per panel of an expanded box: node polynomials (V and K) and the contraction with
        // every used column
        prof::Scope sc(fp64 ? "p2m64" : "p2m", s,
                       double(g.mom_panels) * (8.0 * g.K * NF + 2.0 * NF * 2 * nc),
                       double(g.mom_panels) * 2 * c.pad * esz + mom_bytes);
        if (!launch_p2m_tiles(g, c, dens, mom, s)) {
            switch (g.P) {
                case 2: launch_p2m_p<T, 2>(g, c.pad, dens, mom, s); break;
                case 4: launch_p2m_p<T, 4>(g, c.pad, dens, mom, s); break;
                case 6: launch_p2m_p<T, 6>(g, c.pad, dens, mom, s); break;
                case 8: launch_p2m_p<T, 8>(g, c.pad, dens, mom, s); break;
                case 10: launch_p2m_p<T, 10>(g, c.pad, dens, mom, s); break;
                default: throw Error(LSPR_E_INVALID, "expansion orders above 10 run only from matrix-core tiles");
            }
        }
    }
    {
        // executed work: 2 flops per used column of each operator and pair (direct: kernel
        // value times density; expansion: per Taylor term, coefficient times moment).  The
        // vector-ALU kernel also forms the kernel values (per node 15 flops: difference, r^2,
        // rsqrt, two weighted sums; 9 per pair: centroid difference, plane height, product) and
        // the coefficients (about 10 flops per term of the recurrence); on matrix cores those
        // are geometry-only factors computed once at set-up, and the launch reads them instead
        // (the tile store, once).
        const bool pre = c.mfma && tiles_of<T>(g) != nullptr;
        const double f = double(g.p2p_pairs) * (4.0 * nc + (pre ? 0.0 : 15.0 * g.K + 9.0)) +
                         double(g.m2p_pairs) * g.n_terms * (4.0 * nc + (pre ? 0.0 : 10.0));
        const double tile_bytes = pre ? double(g.tile_elems) * esz : 0.0;
        prof::Scope sc(fp64 ? "far64" : "far", s, f,
                       tile_bytes + dens_bytes + mom_bytes + out_bytes,
                       (double(g.p2p_pairs) * g.K + double(g.m2p_pairs)) * (nc / 2),
                       c.ncol / 2);
        if (c.mfma) {
            LSPR_REQUIRE(tiles_of<T>(g) != nullptr || (g.n_m2p == 0 && g.n_p2p == 0),
                         LSPR_E_INVALID, "matrix-core tiles were not built");
            launch_far_tiles<T>(g, c.pad, dens, mom, os, oa, s);
        } else {
            switch (c.cpt) {
                case 2: launch_far_cpt<T, 2>(g, c.pad, dens, mom, os, oa, s); break;
                case 4: launch_far_cpt<T, 4>(g, c.pad, dens, mom, os, oa, s); break;
                case 16: launch_far_cpt<T, 16>(g, c.pad, dens, mom, os, oa, s); break;
                default: throw Error(LSPR_E_INVALID, "unsupported column blocking");
            }
        }
    }
    if (c.mfma && (fp64 ? g.near_in_tiles64 : g.near_in_tiles32)) return;
    const int64_t tot = static_cast<int64_t>(g.N) * 2 * c.pad;
    prof::Scope sc("near", s, double(g.n_near + g.N) * 2.0 * 2 * nc,
                   double(g.n_near) * 20 + dens_bytes + 2 * out_bytes);
    hipLaunchKernelGGL(k_near_corr<T>, dim3((tot + 255) / 256), dim3(256), 0, s,
                       g.near_off64.p, g.near_col.p, g.near_dv.p, g.near_dk.p, g.vself.p,
                       g.surf.p, g.N, dens, c.pad, os, oa);
    LSPR_HIP(hipGetLastError());
}

template <class T, int P>
void launch_build_m2p(Geometry& g, T* A, float* A32, const TileDesc* tiles, const int32_t* mt,
                      const int32_t* mc, int n, hipStream_t s) {
    hipLaunchKernelGGL((k_build_m2p_tiles<T, P>), dim3(n), dim3(64), 0, s, g.chunks.p,
                       g.boxes.p, tiles, mt, mc, g.m2p_box.p, n, g.cen.p, A, A32);
    LSPR_HIP(hipGetLastError());
}

// Builds the tiles in precision T; A32 (T = double, may be null): the FP32 store, filled with
// the same values rounded.
template <class T>
void build_tiles_t(Geometry& g, T* A, float* A32, const int32_t* mt, const int32_t* mc,
                   int n_m2p, const int32_t* pt, const int32_t* pc, int n_p2p, hipStream_t s) {
    if (n_m2p > 0) {
        switch (g.P) {
            case 2: launch_build_m2p<T, 2>(g, A, A32, g.tiles.p, mt, mc, n_m2p, s); break;
            case 4: launch_build_m2p<T, 4>(g, A, A32, g.tiles.p, mt, mc, n_m2p, s); break;
            case 6: launch_build_m2p<T, 6>(g, A, A32, g.tiles.p, mt, mc, n_m2p, s); break;
            case 8: launch_build_m2p<T, 8>(g, A, A32, g.tiles.p, mt, mc, n_m2p, s); break;
            case 10: launch_build_m2p<T, 10>(g, A, A32, g.tiles.p, mt, mc, n_m2p, s); break;
            case 12: launch_build_m2p<T, 12>(g, A, A32, g.tiles.p, mt, mc, n_m2p, s); break;
            case 15: launch_build_m2p<T, 15>(g, A, A32, g.tiles.p, mt, mc, n_m2p, s); break;
            default: throw Error(LSPR_E_INVALID, "expansion order must be 2, 4, 6, 8, 10, 12 or 15");
        }
    }
    if (n_p2p > 0) {
        LSPR_REQUIRE(4 * direct_steps(g.n_terms) <= P2P_MAXP && 4 + 4 * g.K <= P2P_MAXR,
                     LSPR_E_INVALID, "direct tile larger than the tile builder's staging");
        hipLaunchKernelGGL(k_build_p2p_tiles<T>, dim3(n_p2p), dim3(256), 0, s, g.chunks.p,
                           g.tiles.p, pt, pc, n_p2p, g.cen.p, src_of<T>(g), g.K, A, A32);
        LSPR_HIP(hipGetLastError());
    }
}

}  // namespace

// Folds the near-field terms into freshly built direct tiles; false (and the tiles rebuilt
// without them, so the separate near pass applies) if some pair had no tile.
template <class T>
bool fold_near(Geometry& g, T* A, float* A32, const int32_t* dt_off, const int32_t* dt_row0,
               const int32_t* dt_tile, hipStream_t s,
               const std::function<void()>& rebuild) {
    if (g.N == 0 || g.n_chunks == 0) return false;
    DevBuf<int32_t> miss(1);
    LSPR_HIP(hipMemsetAsync(miss.p, 0, sizeof(int32_t), s));
    const int64_t n_fold = g.n_near + g.N;  // near-singular entries, then the self pairs
    hipLaunchKernelGGL(k_fold_near<T>, dim3(static_cast<unsigned>((n_fold + 255) / 256)), dim3(256),
                       0, s, g.chunks.p, g.n_chunks, dt_off, dt_row0, dt_tile, g.tiles.p,
                       g.near_off64.p, g.near_col.p, g.near_dv.p, g.near_dk.p, g.vself.p, g.N,
                       static_cast<int64_t>(g.n_near), A, A32, miss.p);
    LSPR_HIP(hipGetLastError());
    int32_t h = 0;
    copy_sync(&h, miss.p, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (h == 0) return true;
    rebuild();
    return false;
}

int64_t estimate_tile_elems(const Geometry& g) {
    const int nc = g.n_chunks;
    const int64_t exp_elems = static_cast<int64_t>(expansion_slices(g.n_terms)) *
                              expansion_slice_steps(g.n_terms) * 256;
    int64_t e = static_cast<int64_t>(g.m2p_off_h.size() == static_cast<size_t>(nc) + 1
                                         ? g.m2p_off_h[nc] : 0) * exp_elems;
    const int dmax = direct_steps(g.n_terms);
    for (const Range& r : g.p2p_rng_h) {
        const int n = r.end - r.start, full = n / (4 * dmax), rest = n % (4 * dmax);
        e += (static_cast<int64_t>(full) * dmax + (rest + 3) / 4) * 2 * 256;
    }
    return e;
}

// Work items of the far-field kernels over one tile list (per chunk: first tile `off`, own-
// surface tiles `self`; a tile costs its K-steps + 4).  A chunk whose cost exceeds `split` x the
// mean is cut at its own-surface boundary and into pieces of about equal cost (split 0: whole
// chunks).  The items, in chunk order, are dealt to 8 XCD runs of consecutive items at equal
// shares of the cost, the heaviest first within each run (workgroup b takes an item of run
// b % 8).  A run ends when its last items end, and items that start late leave the other
// slots of the XCD idle until they finish; so the items making up the last `tail` share of
// each run's cost are cut again, into pieces of at most a quarter of the first limit, which the
// ordering puts at the end of the run.  With `cut_self` every chunk that has tiles on both
// sides of its own-surface boundary is cut there too, so no item spans it.  A chunk of several
// items has consecutive partial-sum slots in tile order (own-surface pieces first), added in
// that order by k_far_reduce.
void plan_items(const std::vector<TileDesc>& tl, const std::vector<int32_t>& off,
                const std::vector<int32_t>& self, double split, double tail, bool cut_self,
                TilePlan::Items& W) {
    W.items.clear();
    W.red.clear();
    W.n_slots = 0;
    const int nc = static_cast<int>(self.size());
    auto tcost = [&](int t) { return static_cast<double>(tl[t].nstep) + 4.0; };
    auto rcost = [&](int t0, int t1) {
        double cs = 0.0;
        for (int t = t0; t < t1; ++t) cs += tcost(t);
        return cs;
    };
    double total = 0.0;
    for (int c = 0; c < nc; ++c) total += rcost(off[c], off[c + 1]);
    const double cap = nc > 0 ? split * total / nc : 0.0;
    struct Piece {
        int32_t c, t0, t1, run;
        double cost;
    };
    // [x, y) of chunk c into about equal pieces of at most `lim` (appended in tile order)
    auto cut = [&](int c, int x, int y, int run, double lim, std::vector<Piece>& out) {
        const double cs = rcost(x, y);
        const int n = lim > 0.0 ? std::max(1, static_cast<int>(std::ceil(cs / lim))) : 1;
        double acc = 0.0, done = 0.0;
        int start = x, k = 0;
        for (int t = x; t < y; ++t) {
            acc += tcost(t);
            if (k < n - 1 && t + 1 < y && acc >= (k + 1) * cs / n) {
                out.push_back({c, start, t + 1, run, acc - done});
                done = acc;
                start = t + 1;
                ++k;
            }
        }
        out.push_back({c, start, y, run, acc - done});
    };
    // the cut of a chunk's tiles [x, y) at its own-surface boundary and then by `lim`
    auto cut_chunk = [&](int c, int x, int y, int run, double lim, std::vector<Piece>& out) {
        const int m = off[c] + self[c];
        if ((lim <= 0.0 || rcost(x, y) <= lim) && !(cut_self && x < m && m < y)) {
            out.push_back({c, x, y, run, rcost(x, y)});
            return;
        }
        if (x < m) cut(c, x, std::min(m, y), run, lim, out);
        if (std::max(x, m) < y) cut(c, std::max(x, m), y, run, lim, out);
    };
    std::vector<Piece> pcs;
    for (int c = 0; c < nc; ++c) cut_chunk(c, off[c], off[c + 1], 0, cap, pcs);
    // XCD runs of consecutive items at equal shares of the cost
    {
        const int ni = static_cast<int>(pcs.size());
        double acc = 0.0;
        int x = 0, in_run = 0;
        for (int i = 0; i < ni; ++i) {
            while (x < 7 && in_run > 0 &&
                   (acc + 0.5 * pcs[i].cost > (x + 1) * total / 8.0 || ni - i <= 7 - x)) {
                ++x;
                in_run = 0;
            }
            pcs[i].run = x;
            ++in_run;
            acc += pcs[i].cost;
        }
    }
    auto by_cost = [&](const std::vector<Piece>& v, int run) {
        std::vector<int32_t> ix;
        for (int i = 0; i < static_cast<int>(v.size()); ++i)
            if (v[i].run == run) ix.push_back(i);
        std::stable_sort(ix.begin(), ix.end(),
                         [&](int32_t u, int32_t w) { return v[u].cost > v[w].cost; });
        return ix;
    };
    // the tail of each run cut finer
    if (tail > 0.0 && cap > 0.0) {
        std::vector<char> fine(pcs.size(), 0);
        for (int r = 0; r < 8; ++r) {
            const std::vector<int32_t> ix = by_cost(pcs, r);
            double rc = 0.0, acc = 0.0;
            for (int32_t i : ix) rc += pcs[i].cost;
            for (int k = static_cast<int>(ix.size()) - 1; k >= 0 && acc < tail * rc; --k) {
                fine[ix[k]] = 1;
                acc += pcs[ix[k]].cost;
            }
        }
        std::vector<Piece> ref;
        for (size_t i = 0; i < pcs.size(); ++i) {
            if (fine[i])
                cut_chunk(pcs[i].c, pcs[i].t0, pcs[i].t1, pcs[i].run, 0.25 * cap, ref);
            else
                ref.push_back(pcs[i]);
        }
        pcs.swap(ref);
    }
    // slots: the items of a chunk are consecutive in `pcs`, in tile order
    for (size_t i = 0; i < pcs.size();) {
        size_t j = i + 1;
        while (j < pcs.size() && pcs[j].c == pcs[i].c) ++j;
        const int c = pcs[i].c, m = off[c] + self[c];
        if (j - i == 1) {
            W.items.push_back({c, pcs[i].t0, pcs[i].t1, -1});
        } else {
            FarRed R{c, W.n_slots, 0, 0};
            for (size_t k = i; k < j; ++k) {
                W.items.push_back({c, pcs[k].t0, pcs[k].t1, W.n_slots++});
                if (pcs[k].t1 <= m) ++R.nself;
            }
            R.slot1 = W.n_slots;
            W.red.push_back(R);
        }
        i = j;
    }
    size_t per = 0;
    std::vector<std::vector<int32_t>> runs(8);
    for (int r = 0; r < 8; ++r) {
        runs[r] = by_cost(pcs, r);
        per = std::max(per, runs[r].size());
    }
    W.order.assign(std::max<size_t>(per, 1) * 8, -1);
    for (int r = 0; r < 8; ++r)
        for (size_t i = 0; i < runs[r].size(); ++i) W.order[i * 8 + r] = runs[r][i];
}

namespace {
std::mutex plan_mu;
std::vector<std::unique_ptr<TilePlan>> plan_cache;  // at most 4 kept
}  // namespace

std::unique_ptr<TilePlan> take_plan() {
    std::lock_guard<std::mutex> lk(plan_mu);
    if (plan_cache.empty()) return std::make_unique<TilePlan>();
    std::unique_ptr<TilePlan> p = std::move(plan_cache.back());
    plan_cache.pop_back();
    return p;
}

void put_plan(std::unique_ptr<TilePlan> p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(plan_mu);
    if (plan_cache.size() < 4) plan_cache.push_back(std::move(p));
}

void plan_tiles(const Geometry& g, TilePlan& P) {
    const int nc = g.n_chunks;
    // the lists as the list builder left them on the host
    const std::vector<int32_t>&mo = g.m2p_off_h, &po = g.p2p_off_h, &ms = g.m2p_self_h,
                                &ps = g.p2p_self_h, &mbox = g.m2p_box_h;
    const std::vector<Range>& rng = g.p2p_rng_h;
    LSPR_REQUIRE(static_cast<int>(mo.size()) == nc + 1 && static_cast<int>(po.size()) == nc + 1 &&
                     static_cast<int>(ms.size()) == nc && static_cast<int>(ps.size()) == nc &&
                     static_cast<int64_t>(mbox.size()) == g.n_m2p &&
                     static_cast<int64_t>(rng.size()) == g.n_p2p &&
                     static_cast<int>(g.mom_slot_h.size()) == g.n_boxes,
                 LSPR_E_INVALID, "interaction lists missing on the host");
    const int nsl = expansion_slices(g.n_terms);      // tiles per expansion
    const int nsm = expansion_slice_steps(g.n_terms);  // K-steps of each
    const int dmax = direct_steps(g.n_terms);         // most K-steps of a direct tile
    auto make_tile = [](int kind, int nstep, int64_t aoff, int r0, int rows) {
        LSPR_REQUIRE(aoff % 256 == 0 && aoff / 256 < INT32_MAX, LSPR_E_INVALID,
                     "tile store offset out of range");
        TileDesc T;
        T.kind = static_cast<int16_t>(kind);
        T.nstep = static_cast<int16_t>(nstep);
        T.a_blk = static_cast<int32_t>(aoff / 256);
        T.b_row0 = r0;
        T.b_rows = rows;
        return T;
    };
    std::vector<TileDesc>& tiles = P.tiles;
    std::vector<int32_t>&toff = P.toff, &tself = P.tself, &m2p_tile = P.m2p_tile,
                         &m2p_chunk = P.m2p_chunk, &p2p_tile = P.p2p_tile, &p2p_chunk = P.p2p_chunk;
    toff.assign(nc + 1, 0);
    tself.assign(nc, 0);
    m2p_tile.assign(g.n_m2p, 0);
    m2p_chunk.assign(g.n_m2p, 0);
    tiles.clear();
    p2p_tile.clear();
    p2p_chunk.clear();
    P.aoff = 0;
    {
        int64_t nd = 0;  // direct tiles
        for (const Range& r : rng) nd += (r.end - r.start + 4 * dmax - 1) / (4 * dmax);
        tiles.reserve(static_cast<size_t>(g.n_m2p * nsl + nd));
        p2p_tile.reserve(static_cast<size_t>(nd));
        p2p_chunk.reserve(static_cast<size_t>(nd));
    }
    int64_t& aoff = P.aoff;
    for (int c = 0; c < nc; ++c) {
        toff[c] = static_cast<int32_t>(tiles.size());
        for (int phase = 0; phase < 2; ++phase) {
            const int ma = phase == 0 ? mo[c] : mo[c] + ms[c], mb = phase == 0 ? mo[c] + ms[c] : mo[c + 1];
            const int pa = phase == 0 ? po[c] : po[c] + ps[c], pb = phase == 0 ? po[c] + ps[c] : po[c + 1];
            for (int e = ma; e < mb; ++e) {
                m2p_tile[e] = static_cast<int32_t>(tiles.size());  // its first slice
                m2p_chunk[e] = c;
                for (int k = 0; k < nsl; ++k) {
                    const int t0 = 4 * nsm * k;
                    tiles.push_back(make_tile(0, nsm, aoff,
                                              g.mom_slot_h[mbox[e]] * g.n_terms + t0,
                                              std::min(4 * nsm, g.n_terms - t0)));
                    aoff += static_cast<int64_t>(nsm) * 256;
                }
            }
            for (int e = pa; e < pb; ++e)
                for (int p0 = rng[e].start; p0 < rng[e].end; p0 += 4 * dmax) {
                    const int rows = std::min(4 * dmax, rng[e].end - p0), ns = (rows + 3) / 4;
                    p2p_tile.push_back(static_cast<int32_t>(tiles.size()));
                    p2p_chunk.push_back(c);
                    tiles.push_back(make_tile(1, ns, aoff, p0, rows));
                    aoff += 2 * static_cast<int64_t>(ns) * 256;
                }
            if (phase == 0) tself[c] = static_cast<int32_t>(tiles.size()) - toff[c];
        }
    }
    toff[nc] = static_cast<int32_t>(tiles.size());
    P.tile_steps = 0;
    P.max_chunk_steps = 0;
    std::vector<int64_t> csteps(nc, 0);
    for (int c = 0; c < nc; ++c) {
        for (int t = toff[c]; t < toff[c + 1]; ++t) csteps[c] += tiles[t].nstep;
        P.tile_steps += csteps[c];
        P.max_chunk_steps = std::max(P.max_chunk_steps, csteps[c]);
    }
    // Workgroup order: run x = b % 8 of consecutive chunks (the workgroups of one XCD), the runs
    // cut at equal shares of the estimated work (K-steps plus 4 per tile for its fixed costs),
    // heaviest chunk first within each run.
    std::vector<double> ccost(nc);
    double total = 0.0;
    for (int c = 0; c < nc; ++c) {
        ccost[c] = static_cast<double>(csteps[c]) + 4.0 * (toff[c + 1] - toff[c]);
        total += ccost[c];
    }
    std::vector<std::vector<int32_t>> runs(8);
    {
        double acc = 0.0;
        int x = 0;
        for (int c = 0; c < nc; ++c) {
            // move on to the next run once this one holds its share (every run gets a chunk
            // while enough remain)
            while (x < 7 && !runs[x].empty() &&
                   (acc + 0.5 * ccost[c] > (x + 1) * total / 8.0 || nc - c <= 7 - x))
                ++x;
            runs[x].push_back(c);
            acc += ccost[c];
        }
    }
    size_t per_xcd = 0;
    for (auto& run : runs) {
        std::stable_sort(run.begin(), run.end(),
                         [&](int32_t a, int32_t b) { return ccost[a] > ccost[b]; });
        per_xcd = std::max(per_xcd, run.size());
    }
    std::vector<int32_t>& order = P.order;
    order.assign(std::max<size_t>(per_xcd, 1) * 8, -1);
    for (int x = 0; x < 8; ++x)
        for (size_t i = 0; i < runs[x].size(); ++i) order[i * 8 + x] = runs[x][i];
    // Work items per launch class (planned once for classes of equal parameters); no item spans
    // a chunk's own-surface boundary (k_far_wide needs it).
    for (int cls = 0; cls < 3; ++cls) {
        int same = -1;
        for (int k = 0; k < cls && same < 0; ++k)
            if (g.far_split[k] == g.far_split[cls] && g.far_tail[k] == g.far_tail[cls]) same = k;
        if (same >= 0)
            P.far[cls] = P.far[same];
        else
            plan_items(tiles, toff, tself, g.far_split[cls], g.far_tail[cls], true, P.far[cls]);
    }
    // each chunk's direct tiles sorted by first source panel, for the near-field fold
    P.dto.assign(nc + 1, 0);
    P.dtr.clear();
    P.dti.clear();
    P.dtr.reserve(p2p_tile.size());
    P.dti.reserve(p2p_tile.size());
    std::vector<std::pair<int32_t, int32_t>> d;
    for (int c = 0; c < nc; ++c) {
        P.dto[c] = static_cast<int32_t>(P.dti.size());
        d.clear();
        for (int t = toff[c]; t < toff[c + 1]; ++t)
            if (tiles[t].kind == 1) d.emplace_back(tiles[t].b_row0, t);
        std::sort(d.begin(), d.end());
        for (auto& e : d) {
            P.dtr.push_back(e.first);
            P.dti.push_back(e.second);
        }
    }
    P.dto[nc] = static_cast<int32_t>(P.dti.size());
}

void build_tiles(Geometry& g, const TilePlan& P) {
    hipStream_t s = g.stream;
    const int nc = g.n_chunks;
    LSPR_REQUIRE(static_cast<int>(P.toff.size()) == nc + 1, LSPR_E_INVALID,
                 "tile plan does not match the geometry");
    g.tile_steps = P.tile_steps;
    g.max_chunk_steps = P.max_chunk_steps;
    g.tile_elems = P.aoff;
    const std::vector<int32_t>& order = P.order;
    const int64_t aoff = P.aoff;
    g.n_order = static_cast<int>(order.size());
    // Tile stores within the budget: FP32 first (the GMRES products of the FP32 and refinement
    // modes), then FP64 with what is left.  A precision without tiles keeps the on-the-fly
    // vector-ALU kernel (e.g. a dense product on a big mesh).
    double left = g.tile_budget_bytes;
    const bool keep32 = g.need32 && static_cast<double>(aoff) * 4.0 <= left;
    if (keep32) left -= static_cast<double>(aoff) * 4.0;
    const bool keep64 = g.need64 && static_cast<double>(aoff) * 8.0 <= left;
    LSPR_REQUIRE(g.P <= 10 || ((!g.need32 || keep32) && (!g.need64 || keep64)), LSPR_E_NOMEM,
                 "expansion orders above 10 run only from matrix-core tiles, and they do not "
                 "fit the tile budget");
    if (!keep32 && !keep64) {
        g.n_tiles = 0;
        return;
    }
    g.n_tiles = static_cast<int64_t>(P.tiles.size());
    g.tiles.alloc(std::max<int64_t>(g.n_tiles, 1));
    g.tile_off.alloc(nc + 1);
    g.tile_self.alloc(nc);
    g.chunk_order.alloc(order.size());
    Uploads up(s);  // every table below in one transfer
    up.add(g.chunk_order.p, order.data(), order.size());
    up.add(g.tiles.p, P.tiles.data(), P.tiles.size());
    up.add(g.tile_off.p, P.toff.data(), P.toff.size());
    up.add(g.tile_self.p, P.tself.data(), P.tself.size());
    for (int cls = 0; cls < 3; ++cls) {
        Geometry::FarPlan& fp = g.far_plan[cls];
        const TilePlan::Items& W = P.far[cls];
        fp.items.alloc(W.items.size());
        fp.order.alloc(W.order.size());
        up.add(fp.items.p, W.items.data(), W.items.size());
        up.add(fp.order.p, W.order.data(), W.order.size());
        fp.n_order = static_cast<int>(W.order.size());
        fp.n_red = static_cast<int>(W.red.size());
        fp.n_slots = W.n_slots;
        if (!W.red.empty()) {
            fp.red.alloc(W.red.size());
            up.add(fp.red.p, W.red.data(), W.red.size());
        }
    }
    const int n_m2p = static_cast<int>(g.n_m2p), n_p2p = static_cast<int>(P.p2p_tile.size());
    DevBuf<int32_t> mt(n_m2p), mc(n_m2p), pt(n_p2p), pc(n_p2p);
    up.add(mt.p, P.m2p_tile.data(), n_m2p);
    up.add(mc.p, P.m2p_chunk.data(), n_m2p);
    up.add(pt.p, P.p2p_tile.data(), n_p2p);
    up.add(pc.p, P.p2p_chunk.data(), n_p2p);
    DevBuf<int32_t> dto_d(nc + 1), dtr_d(std::max<size_t>(P.dtr.size(), 1)), dti_d(std::max<size_t>(P.dti.size(), 1));
    up.add(dto_d.p, P.dto.data(), P.dto.size());
    up.add(dtr_d.p, P.dtr.data(), P.dtr.size());
    up.add(dti_d.p, P.dti.data(), P.dti.size());
    up.flush();
    if (keep32) g.tileA.alloc(std::max<int64_t>(aoff, 1));
    if (keep64) g.tileA64.alloc(std::max<int64_t>(aoff, 1));
    // the moments' tiles, for each precision with tiles, on a second stream beside the expansion
    // and direct tiles (a latency-bound builder next to two bandwidth-bound ones)
    struct AuxStream {
        hipStream_t s = nullptr;
        ~AuxStream() {
            if (s) {
                (void)hipStreamSynchronize(s);
                (void)hipStreamDestroy(s);
            }
        }
    } aux;
    if (g.n_seg > 0) {
        LSPR_HIP(hipStreamCreateWithFlags(&aux.s, hipStreamNonBlocking));
        switch (g.P) {
            case 2: build_p2m_tiles_p<2>(g, s, aux.s); break;
            case 4: build_p2m_tiles_p<4>(g, s, aux.s); break;
            case 6: build_p2m_tiles_p<6>(g, s, aux.s); break;
            case 8: build_p2m_tiles_p<8>(g, s, aux.s); break;
            case 10: build_p2m_tiles_p<10>(g, s, aux.s); break;
            case 12: build_p2m_tiles_p<12>(g, s, aux.s); break;
            case 15: build_p2m_tiles_p<15>(g, s, aux.s); break;
            default: throw Error(LSPR_E_INVALID, "expansion order must be 2, 4, 6, 8, 10, 12 or 15");
        }
    }
    // with both stores, one FP64 pass fills both (the FP32 tiles are the FP64 values rounded)
    if (keep64) {
        float* a32 = keep32 ? g.tileA.p : nullptr;
        auto build = [&] { build_tiles_t<double>(g, g.tileA64.p, a32, mt.p, mc.p, n_m2p, pt.p, pc.p, n_p2p, s); };
        build();
        g.near_in_tiles64 = fold_near(g, g.tileA64.p, a32, dto_d.p, dtr_d.p, dti_d.p, s, build);
        if (keep32) g.near_in_tiles32 = g.near_in_tiles64;
    } else if (keep32) {
        auto build = [&] { build_tiles_t<float>(g, g.tileA.p, nullptr, mt.p, mc.p, n_m2p, pt.p, pc.p, n_p2p, s); };
        build();
        g.near_in_tiles32 = fold_near(g, g.tileA.p, nullptr, dto_d.p, dtr_d.p, dti_d.p, s, build);
    }
    LSPR_HIP(hipStreamSynchronize(s));
    if (aux.s) LSPR_HIP(hipStreamSynchronize(aux.s));
}

Cols make_cols(const Geometry& g, int ncol, int prec) {
    Cols c;
    c.ncol = ncol;
    c.prec = prec;
    const bool tiles = prec == LSPR_FP32 ? g.tileA.p != nullptr : g.tileA64.p != nullptr;
    if (g.allow_mfma && (tiles || g.n_chunks == 0)) {
        // matrix cores from precomputed tiles: 16 K columns (and 16 V columns) per wavefront;
        // the tile stream dominates, so even a single wavelength is cheapest this way
        c.mfma = true;
        c.cpt = 16;
        c.pad = (ncol + 15) / 16 * 16;
        LSPR_REQUIRE(c.pad / 16 * 64 <= 512, LSPR_E_INVALID,
                     "too many columns in one product (at most 64 wavelengths)");
        return c;
    }
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
    if (c.prec == LSPR_FP32)
        apply_far_t<float>(g, c, static_cast<const float*>(dens), os, out_all, s);
    else
        apply_far_t<double>(g, c, static_cast<const double*>(dens), os, out_all, s);
}

}  // namespace lspr
