// Octree, interaction lists, near-singular correction table and singular self-terms
// (set-up, once per mesh and parameter set).
//
// Section "Acceleration strategies": sources are grouped in the boxes of an octree whose
// leaves hold at most N_crit sources; a target uses a box's Taylor expansion when the box is
// far enough (MAC theta > r_b / r, r measured from the box centre), opens it otherwise, and
// sums a leaf that is still too close directly.  Here the targets of a group of consecutive
// panels (a "chunk") share their lists: a box is accepted for the whole chunk when
// r_b < theta (d - r_T) (d the centre distance, r_T the chunk radius), which implies the
// paper's per-target criterion for every target of the chunk.  Section "Integral evaluation":
// near-singular pairs (|x_i - c_j| <= L_j / threshold) and the singular self pair use other
// rules; the table built here holds, per such pair, the fine-rule value minus the far-rule
// value that the direct sum adds, so that the far-field kernels can treat all pairs alike.
#include <cmath>

#include "primitives.hpp"

namespace lspr {

namespace {

constexpr int TPB = 256;
constexpr int MAX_LEVEL = 16;   // 16 Morton bits per axis

__device__ inline void node_pos(const double* v, const double* rule, int g, double* y) {
    const double b0 = rule[4 * g], b1 = rule[4 * g + 1], b2 = rule[4 * g + 2];
    for (int d = 0; d < 3; ++d) y[d] = b0 * v[d] + b1 * v[3 + d] + b2 * v[6 + d];
}

template <class Op>
__device__ inline double block_reduce(double v, double* sh, Op op) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = op(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

struct MinOp { __device__ double operator()(double a, double b) const { return fmin(a, b); } };
struct MaxOp { __device__ double operator()(double a, double b) const { return fmax(a, b); } };

// Boxes of more panels than this get blocks of 1024 threads (a launch of their own).
constexpr int BIG_BOX = 2048;

// One block of NT threads per box: centre of the nodes' bounding box, node radius, vertex radius,
// max L.  With `list` the blocks take the listed boxes; without it, every box of at most
// BIG_BOX panels (the others are in the list).
template <int NT>
__global__ void __launch_bounds__(NT) k_box_stats(Box* __restrict__ boxes,
                                                  const int32_t* __restrict__ list,
                                                  const double* __restrict__ tri,
                                                  const double* __restrict__ area,
                                                  const double* __restrict__ rule, int K) {
    __shared__ double sh[NT];
    Box& b = boxes[list != nullptr ? list[blockIdx.x] : blockIdx.x];
    const int start = b.start, end = b.end;
    if (list == nullptr && end - start > BIG_BOX) return;  // whole block: the box is listed
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int p = start + threadIdx.x; p < end; p += NT) {
        const double* v = tri + 9 * static_cast<size_t>(p);
        for (int gq = 0; gq < K; ++gq) {
            double y[3];
            node_pos(v, rule, gq, y);
            for (int d = 0; d < 3; ++d) {
                lo[d] = fmin(lo[d], y[d]);
                hi[d] = fmax(hi[d], y[d]);
            }
        }
    }
    double c[3];
    for (int d = 0; d < 3; ++d)
        c[d] = 0.5 * (block_reduce(lo[d], sh, MinOp()) + block_reduce(hi[d], sh, MaxOp()));
    double rb = 0.0, rv = 0.0, lm = 0.0;
    for (int p = start + threadIdx.x; p < end; p += NT) {
        const double* v = tri + 9 * static_cast<size_t>(p);
        for (int gq = 0; gq < K; ++gq) {
            double y[3];
            node_pos(v, rule, gq, y);
            const double dx = y[0] - c[0], dy = y[1] - c[1], dz = y[2] - c[2];
            rb = fmax(rb, sqrt(dx * dx + dy * dy + dz * dz));
        }
        for (int k = 0; k < 3; ++k) {
            const double dx = v[3 * k] - c[0], dy = v[3 * k + 1] - c[1], dz = v[3 * k + 2] - c[2];
            rv = fmax(rv, sqrt(dx * dx + dy * dy + dz * dz));
        }
        lm = fmax(lm, sqrt(2.0 * area[p]));
    }
    rb = block_reduce(rb, sh, MaxOp());
    rv = block_reduce(rv, sh, MaxOp());
    lm = block_reduce(lm, sh, MaxOp());
    if (threadIdx.x == 0) {
        b.cx = c[0];
        b.cy = c[1];
        b.cz = c[2];
        b.rb = rb;
        b.rv = rv;
        b.lmax = lm;
    }
}

// One block per chunk: centre of the centroids' bounding box and radius.
__global__ void __launch_bounds__(TPB) k_chunk_stats(Chunk* __restrict__ ch,
                                                     const double* __restrict__ cen) {
    __shared__ double sh[TPB];
    Chunk& c = ch[blockIdx.x];
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int p = c.start + threadIdx.x; p < c.end; p += TPB)
        for (int d = 0; d < 3; ++d) {
            lo[d] = fmin(lo[d], cen[3 * p + d]);
            hi[d] = fmax(hi[d], cen[3 * p + d]);
        }
    double m[3];
    for (int d = 0; d < 3; ++d)
        m[d] = 0.5 * (block_reduce(lo[d], sh, MinOp()) + block_reduce(hi[d], sh, MaxOp()));
    double r = 0.0;
    for (int p = c.start + threadIdx.x; p < c.end; p += TPB) {
        const double dx = cen[3 * p] - m[0], dy = cen[3 * p + 1] - m[1], dz = cen[3 * p + 2] - m[2];
        r = fmax(r, sqrt(dx * dx + dy * dy + dz * dz));
    }
    r = block_reduce(r, sh, MaxOp());
    if (threadIdx.x == 0) {
        c.cx = m[0];
        c.cy = m[1];
        c.cz = m[2];
        c.r = r;
    }
}

struct ListParams {
    double theta, inv_thr;
    int min_panels;
    int S;
    const int32_t* roots;  // [S]
};

// Interaction lists of one chunk against every surface's tree, own surface first.  A box is
// expanded (M2P) when the MAC holds for the whole chunk, no target of the chunk can be
// near-singular to any of its panels (d - r_T - r_v > L_max / threshold), and it holds enough
// panels for the expansion to be cheaper than the direct sum; otherwise a leaf, or a box that
// passes the MAC but is small, is summed directly; any other box is opened.  Direct ranges that
// touch are merged.  The lists are those of one depth-first walk per (chunk, surface); the walk
// is split over up to SUBS sub-trees (the boxes two levels below the root, in depth-first
// order, or a shallower box that is not opened), one thread each: a count pass, a per-chunk pass
// that places the sub-lists and merges direct ranges across sub-tree boundaries, and a fill pass.
constexpr int SUBS = 64;
enum ListAction { LIST_OPEN = 0, LIST_M2P = 1, LIST_P2P = 2 };

__device__ __forceinline__ int list_action(const Chunk& T, const Box& B, const ListParams& lp) {
    const double dx = T.cx - B.cx, dy = T.cy - B.cy, dz = T.cz - B.cz;
    const double d = sqrt(dx * dx + dy * dy + dz * dz);
    const bool ok = d > T.r && B.rb < lp.theta * (d - T.r) &&
                    (d - T.r - B.rv) > B.lmax * lp.inv_thr;
    if (ok && B.end - B.start >= lp.min_panels) return LIST_M2P;
    if (ok || B.nchild == 0) return LIST_P2P;
    return LIST_OPEN;
}

// Root of sub-tree k of the walk from `root` for chunk T, or -1.
__device__ int sub_root(const Box* __restrict__ boxes, const Chunk& T, int root, int k,
                        const ListParams& lp) {
    const Box R = boxes[root];
    if (list_action(T, R, lp) != LIST_OPEN) return k == 0 ? root : -1;
    int n = 0;
    for (int i = 0; i < R.nchild; ++i) {
        const int ci = R.child + i;
        const Box Cb = boxes[ci];
        if (list_action(T, Cb, lp) != LIST_OPEN) {
            if (n == k) return ci;
            ++n;
        } else {
            if (k < n + Cb.nchild) return Cb.child + (k - n);
            n += Cb.nchild;
        }
    }
    return -1;
}

// One sub-tree's part of the lists.  flags: 1 its first item is a direct range, 2 its last item
// is a direct range, 4 it has items.  first_end: end of its first direct range (after merges).
struct SubList {
    int32_t nm, np, first_end, flags;
    int64_t pp, mp;
};
// Where a sub-tree writes: offsets within the chunk's lists; skip: its first direct range joins
// the previous sub-tree's last one; end: new end of its last direct range (-1: unchanged).
struct SubPlace {
    int32_t m2p, p2p, skip, end;
};

template <bool FILL>
__device__ void walk_sub(const Box* __restrict__ boxes, const Chunk& T, int q,
                         const ListParams& lp, SubList& L, const SubPlace& pl,
                         int32_t* __restrict__ m2p_box, Range* __restrict__ p2p_rng) {
    const int nt = T.end - T.start;
    // depth-first over q's subtree without a stack: into the first child, or past the subtree
    const int stop = boxes[q].next;
    int bi = q;
    int last_end = -1, li = -1;  // li: local index of the last direct range
    auto slot = [&](int i) { return pl.p2p + i - pl.skip; };
    while (bi != stop) {
        const int cur = bi;
        const Box B = boxes[cur];
        const int act = list_action(T, B, lp);
        bi = B.next;
        if (act == LIST_M2P) {
            if (FILL) m2p_box[pl.m2p + L.nm] = cur;
            ++L.nm;
            L.mp += nt;
            L.flags = (L.flags & ~2) | 4;
        } else if (act == LIST_P2P) {
            if (!(L.flags & 4)) L.flags |= 1;
            if (B.start == last_end) {
                if (FILL && !(pl.skip && li == 0)) p2p_rng[slot(li)].end = B.end;
            } else {
                ++li;
                ++L.np;
                if (FILL && !(pl.skip && li == 0)) p2p_rng[slot(li)] = Range{B.start, B.end};
            }
            if (li == 0) L.first_end = B.end;
            last_end = B.end;
            L.pp += static_cast<int64_t>(nt) * (B.end - B.start);
            L.flags |= 2 | 4;
        } else if (B.nchild > 0) {
            bi = B.child;
        }
    }
    if (FILL && pl.end >= 0 && (L.flags & 2) && !(pl.skip && li == 0)) p2p_rng[slot(li)].end = pl.end;
}

__device__ __forceinline__ void list_task(int t, int n_chunks, const ListParams& lp, int& c,
                                          int& pass, int& k) {
    k = t % SUBS;
    pass = (t / SUBS) % lp.S;
    c = t / (SUBS * lp.S);
}

__global__ void k_lists_count(const Box* __restrict__ boxes, const Chunk* __restrict__ chunks,
                              int n_chunks, ListParams lp, SubList* __restrict__ sub) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(n_chunks) * lp.S * SUBS) return;
    int c, pass, k;
    list_task(static_cast<int>(t), n_chunks, lp, c, pass, k);
    const Chunk T = chunks[c];
    const int s = pass == 0 ? T.surf : (pass <= T.surf ? pass - 1 : pass);
    SubList L{0, 0, -1, 0, 0, 0};
    const int q = sub_root(boxes, T, lp.roots[s], k, lp);
    if (q >= 0) walk_sub<false>(boxes, T, q, lp, L, SubPlace{0, 0, 0, -1}, nullptr, nullptr);
    sub[t] = L;
}

// One thread per chunk: sub-list offsets in depth-first order, direct ranges merged across
// sub-tree boundaries (within a surface), per-chunk counts.
__global__ void k_lists_place(const SubList* __restrict__ sub, int n_chunks, int S,
                              SubPlace* __restrict__ place, int32_t* __restrict__ m2p_cnt,
                              int32_t* __restrict__ p2p_cnt, int32_t* __restrict__ m2p_selfc,
                              int32_t* __restrict__ p2p_selfc, int64_t* __restrict__ pairs) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_chunks) return;
    int nm = 0, np = 0;
    int64_t pp = 0, mp = 0;
    for (int pass = 0; pass < S; ++pass) {
        int64_t open = -1;  // sub-tree whose last direct range is still open
        for (int k = 0; k < SUBS; ++k) {
            const int64_t t = (static_cast<int64_t>(c) * S + pass) * SUBS + k;
            const SubList L = sub[t];
            SubPlace P{nm, np, 0, -1};
            if (L.flags & 4) {
                const bool join = open >= 0 && (L.flags & 1);
                if (join) {
                    P.skip = 1;
                    place[open].end = L.first_end;
                }
                const bool only_range = L.nm == 0 && L.np == 1;
                if (!(join && only_range)) open = (L.flags & 2) ? t : -1;
                nm += L.nm;
                np += L.np - P.skip;
                pp += L.pp;
                mp += L.mp;
            }
            place[t] = P;
        }
        if (pass == 0) {
            m2p_selfc[c] = nm;
            p2p_selfc[c] = np;
        }
    }
    m2p_cnt[c] = nm;
    p2p_cnt[c] = np;
    pairs[2 * c] = pp;
    pairs[2 * c + 1] = mp;
}

__global__ void k_lists_fill(const Box* __restrict__ boxes, const Chunk* __restrict__ chunks,
                             int n_chunks, ListParams lp, const SubPlace* __restrict__ place,
                             const int64_t* __restrict__ m2p_off, const int64_t* __restrict__ p2p_off,
                             int32_t* __restrict__ m2p_box, Range* __restrict__ p2p_rng) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(n_chunks) * lp.S * SUBS) return;
    int c, pass, k;
    list_task(static_cast<int>(t), n_chunks, lp, c, pass, k);
    const Chunk T = chunks[c];
    const int s = pass == 0 ? T.surf : (pass <= T.surf ? pass - 1 : pass);
    const int q = sub_root(boxes, T, lp.roots[s], k, lp);
    if (q < 0) return;
    SubList L{0, 0, -1, 0, 0, 0};
    walk_sub<true>(boxes, T, q, lp, L, place[t], m2p_box + m2p_off[c], p2p_rng + p2p_off[c]);
}

struct NearParams {
    double inv_thr;
    int S;
    const int32_t* roots;
    int32_t* maxcnt;    // largest count of a target (counting walk)
};

// Near-singular source panels of every target panel, all surfaces, ascending index order.
// Counting walk (fill false): cnt[i], and (slot not null) the first `cap` panels of target i in
// slot[i cap ..]; filling walk: col[off[i] ..].
__global__ void k_near(const Box* __restrict__ boxes, const double* __restrict__ cen,
                       const double* __restrict__ area, int N, NearParams np, bool fill,
                       int64_t* __restrict__ cnt, const int64_t* __restrict__ off,
                       int32_t* __restrict__ col, int32_t* __restrict__ slot, int cap) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double x = cen[3 * i], y = cen[3 * i + 1], z = cen[3 * i + 2];
    int64_t k = fill ? off[i] : 0;
    int n = 0;
    for (int s = 0; s < np.S; ++s) {
        // depth-first without a stack: into the first child, or past the box's subtree
        int bi = np.roots[s];
        while (bi >= 0) {
            const Box B = boxes[bi];
            const double dx = x - B.cx, dy = y - B.cy, dz = z - B.cz;
            const double d = sqrt(dx * dx + dy * dy + dz * dz);
            const bool far = d - B.rv > B.lmax * np.inv_thr * (1.0 + 1e-9) + 1e-12;
            if (!far && B.nchild > 0) {
                bi = B.child;
                continue;
            }
            if (!far) {
                for (int j = B.start; j < B.end; ++j) {
                    if (j == i) continue;
                    const double ex = x - cen[3 * j], ey = y - cen[3 * j + 1], ez = z - cen[3 * j + 2];
                    const double dj = sqrt(ex * ex + ey * ey + ez * ez);
                    if (dj <= sqrt(2.0 * area[j]) * np.inv_thr) {
                        if (fill) col[k + n] = j;
                        else if (slot != nullptr && n < cap) slot[static_cast<size_t>(i) * cap + n] = j;
                        ++n;
                    }
                }
            }
            bi = B.next;
        }
    }
    if (!fill) {
        cnt[i] = n;
        atomicMax(np.maxcnt, n);
    }
}

// The counting walk's slots moved into the table: one wave per target, lane e copies entry e.
__global__ void __launch_bounds__(64) k_near_compact(const int32_t* __restrict__ slot, int cap,
                                                     const int64_t* __restrict__ off,
                                                     int32_t* __restrict__ col) {
    const int i = blockIdx.x, e = threadIdx.x;
    const int64_t o = off[i], n = off[i + 1] - o;
    for (int q = e; q < n; q += 64) col[o + q] = slot[static_cast<size_t>(i) * cap + q];
}

// Rule sums of one panel at point x (no 1/4pi): V = sum w/r, K = sum w n.(x - y)/r^3.
__device__ inline void rule_sums(const double* v, const double* nrm, double A, const double* x,
                                 const double* rule, int K, double& sv, double& sk) {
    sv = 0.0;
    sk = 0.0;
    for (int gq = 0; gq < K; ++gq) {
        double y[3];
        node_pos(v, rule, gq, y);
        const double dx = x[0] - y[0], dy = x[1] - y[1], dz = x[2] - y[2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double r = sqrt(r2);
        const double w = A * rule[4 * gq + 3];
        sv += w / r;
        sk += w * (nrm[0] * dx + nrm[1] * dy + nrm[2] * dz) / (r2 * r);
    }
}

// Fine-rule minus far-rule values for every near-singular pair.
__global__ void k_near_values(const int32_t* __restrict__ row_of, const int32_t* __restrict__ col,
                              int64_t nnz, const double* __restrict__ tri,
                              const double* __restrict__ cen, const double* __restrict__ nrm,
                              const double* __restrict__ area, const double* __restrict__ far_rule,
                              int K, const double* __restrict__ fine_rule, int Kf,
                              double* __restrict__ dv, double* __restrict__ dk) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const int i = row_of[e], j = col[e];
    const double* v = tri + 9 * static_cast<size_t>(j);
    double fv, fk, cv, ck;
    rule_sums(v, nrm + 3 * j, area[j], cen + 3 * i, fine_rule, Kf, fv, fk);
    rule_sums(v, nrm + 3 * j, area[j], cen + 3 * i, far_rule, K, cv, ck);
    dv[e] = fv - cv;
    dk[e] = fk - ck;
}

__global__ void k_row_of(const int64_t* __restrict__ off, int N, int32_t* __restrict__ row_of) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    for (int64_t e = off[i]; e < off[i + 1]; ++e) row_of[e] = i;
}

// Singular self term (section "Integral evaluation"): the panel is split at its centroid into
// three sub-triangles (centroid, edge); for an edge at perpendicular distance h the radial
// integral is exact (the ray at angle a from the perpendicular meets the edge at h / cos a)
// and the angle integral takes n_k Gauss-Legendre nodes.  Result without 1/4pi.
__global__ void k_vself(const double* __restrict__ tri, const double* __restrict__ cen,
                        const double* __restrict__ nrm, int N, const double* __restrict__ gl_t,
                        const double* __restrict__ gl_w, int nk, double* __restrict__ vself) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double* v = tri + 9 * static_cast<size_t>(i);
    const double* n = nrm + 3 * i;
    const double* x = cen + 3 * i;
    double total = 0.0;
    for (int e = 0; e < 3; ++e) {
        const double* a = v + 3 * e;
        const double* b = v + 3 * ((e + 1) % 3);
        const double ex = b[0] - a[0], ey = b[1] - a[1], ez = b[2] - a[2];
        const double len = sqrt(ex * ex + ey * ey + ez * ez);
        const double ux = ex / len, uy = ey / len, uz = ez / len;
        // in-plane direction away from the panel: edge x normal
        const double ox = uy * n[2] - uz * n[1], oy = uz * n[0] - ux * n[2], oz = ux * n[1] - uy * n[0];
        const double ax = a[0] - x[0], ay = a[1] - x[1], az = a[2] - x[2];
        const double bx = b[0] - x[0], by = b[1] - x[1], bz = b[2] - x[2];
        const double h = ax * ox + ay * oy + az * oz;
        const double al = atan2(ax * ux + ay * uy + az * uz, h);
        const double be = atan2(bx * ux + by * uy + bz * uz, h);
        const double half = 0.5 * (be - al), mid = 0.5 * (be + al);
        double s = 0.0;
        for (int k = 0; k < nk; ++k) s += gl_w[k] / cos(mid + half * gl_t[k]);
        total += half * h * s;
    }
    vself[i] = total;
}

std::vector<double> rule_rows(int n) {
    std::vector<double> bary, w;
    LSPR_REQUIRE(triangle_rule(n, bary, w), LSPR_E_INVALID, "unsupported triangle rule");
    std::vector<double> r(4 * n);
    for (int q = 0; q < n; ++q) {
        r[4 * q] = bary[3 * q];
        r[4 * q + 1] = bary[3 * q + 1];
        r[4 * q + 2] = bary[3 * q + 2];
        r[4 * q + 3] = w[q];
    }
    return r;
}

}  // namespace

void build_tree(Geometry& g) {
    hipStream_t s = g.stream;
    // kept per thread between geometries: its capacity (and host pages) are reused
    static thread_local std::vector<Box> bx;
    bx.clear();
    g.surf_root.assign(g.S, 0);
    g.max_depth = 0;
    // The sorted keys are read back once, into a reused pinned buffer, and the octant bounds of
    // the boxes found on the host: a few binary searches per box, instead of a device pass and a
    // round trip per level.
    struct PinnedKeys {
        PinnedBuf b;
        ~PinnedKeys() {
            if (b.p) pinned_put(b);
        }
    } pk;
    pk.b = pinned_take(static_cast<size_t>(g.N) * sizeof(uint64_t));
    try {
        copy_sync(pk.b.p, g.morton.p, static_cast<size_t>(g.N) * sizeof(uint64_t),
                  hipMemcpyDeviceToHost, s);
    } catch (...) {
        (void)hipStreamSynchronize(s);  // no transfer into the buffer once it is put back
        throw;
    }
    const uint64_t* keys = reinterpret_cast<const uint64_t*>(pk.b.p);
    // lower bounds of box b's 8 octants (first index with octant >= o), then its end: the octant
    // bits follow the box's common prefix, so they are sorted inside the box.  The 8 searches run
    // in lockstep without branches: the remaining length halves whatever the keys, so their loads
    // overlap instead of forming one chain.
    auto split_box = [&](const Box& b, int32_t* out) {
        const int shift = 45 - 3 * b.level;
        auto oct = [&](int k) { return static_cast<int>((keys[k] >> shift) & 7); };
        int base[8];
        for (int o = 0; o < 8; ++o) base[o] = b.start;
        int n = b.end - b.start;
        while (n > 1) {  // the bound of o is in [base[o], base[o] + n]
            const int half = n >> 1;
            for (int o = 0; o < 8; ++o) base[o] = oct(base[o] + half) < o ? base[o] + half : base[o];
            n -= half;
        }
        for (int o = 0; o < 8; ++o)
            out[o] = n == 0 ? b.start : base[o] + (oct(base[o]) < o ? 1 : 0);
        out[8] = b.end;
    };
    for (int sf = 0; sf < g.S; ++sf) {
        Box root{};
        root.start = g.surf_start[sf];
        root.end = g.surf_start[sf + 1];
        root.child = -1;
        root.nchild = 0;
        root.level = 0;
        root.surf = sf;
        g.surf_root[sf] = static_cast<int>(bx.size());
        bx.push_back(root);
        std::vector<int> frontier = {g.surf_root[sf]};
        for (int level = 0; level < MAX_LEVEL && !frontier.empty(); ++level) {
            std::vector<int> split;
            for (int b : frontier)
                if (bx[b].end - bx[b].start > g.ncrit) split.push_back(b);
            if (split.empty()) break;
            const int nb = static_cast<int>(split.size());
            std::vector<int32_t> out(9 * nb);
            for (int k = 0; k < nb; ++k) split_box(bx[split[k]], out.data() + 9 * k);
            std::vector<int> next;
            for (int k = 0; k < nb; ++k) {
                const int b = split[k];
                bx[b].child = static_cast<int>(bx.size());
                int nc = 0;
                for (int o = 0; o < 8; ++o) {
                    if (out[9 * k + o] < out[9 * k + o + 1]) {
                        Box c{};
                        c.start = out[9 * k + o];
                        c.end = out[9 * k + o + 1];
                        c.child = -1;
                        c.nchild = 0;
                        c.level = level + 1;
                        c.surf = sf;
                        next.push_back(static_cast<int>(bx.size()));
                        bx.push_back(c);
                        ++nc;
                    }
                }
                bx[b].nchild = nc;
                g.max_depth = std::max(g.max_depth, level + 1);
            }
            frontier.swap(next);
        }
    }
    // depth-first successors: a child is followed by its next sibling, the last child by its
    // parent's successor (boxes are numbered level by level, so a parent's is set first)
    for (Box& b : bx) b.next = -1;
    for (size_t b = 0; b < bx.size(); ++b)
        for (int k = 0; k < bx[b].nchild; ++k)
            bx[bx[b].child + k].next = k + 1 < bx[b].nchild ? bx[b].child + k + 1 : bx[b].next;
    g.n_boxes = static_cast<int>(bx.size());
    g.n_leaves = 0;
    for (const Box& b : bx) g.n_leaves += b.nchild == 0;
    g.box_rng_h.resize(bx.size());
    for (size_t b = 0; b < bx.size(); ++b) g.box_rng_h[b] = Range{bx[b].start, bx[b].end};
    // target chunks: consecutive panels of one surface
    std::vector<Chunk> ch;
    for (int sf = 0; sf < g.S; ++sf)
        for (int a = g.surf_start[sf]; a < g.surf_start[sf + 1]; a += g.tchunk) {
            Chunk c{};
            c.start = a;
            c.end = std::min(a + g.tchunk, g.surf_start[sf + 1]);
            c.surf = sf;
            ch.push_back(c);
        }
    g.n_chunks = static_cast<int>(ch.size());
    g.boxes.alloc(bx.size());
    g.chunks.alloc(ch.size());
    const std::vector<double> rule = rule_rows(g.K);
    g.far_rule.alloc(rule.size());
    std::vector<int32_t> big;  // boxes for the 1024-thread blocks
    for (size_t b = 0; b < bx.size(); ++b)
        if (bx[b].end - bx[b].start > BIG_BOX) big.push_back(static_cast<int32_t>(b));
    DevBuf<int32_t> big_d(std::max<size_t>(big.size(), 1));
    Uploads up(s);
    up.add(g.boxes.p, bx.data(), bx.size());
    up.add(g.chunks.p, ch.data(), ch.size());
    up.add(g.far_rule.p, rule.data(), rule.size());
    up.add(big_d.p, big.data(), big.size());
    up.flush();
    if (!big.empty()) {
        hipLaunchKernelGGL(k_box_stats<1024>, dim3(big.size()), dim3(1024), 0, s, g.boxes.p,
                           big_d.p, g.tri.p, g.area.p, g.far_rule.p, g.K);
        LSPR_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_box_stats<TPB>, dim3(g.n_boxes), dim3(TPB), 0, s, g.boxes.p,
                       static_cast<const int32_t*>(nullptr), g.tri.p, g.area.p, g.far_rule.p,
                       g.K);
    LSPR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_chunk_stats, dim3(g.n_chunks), dim3(TPB), 0, s, g.chunks.p, g.cen.p);
    LSPR_HIP(hipGetLastError());
    LSPR_HIP(hipStreamSynchronize(s));
}

void build_lists(Geometry& g) {
    hipStream_t s = g.stream;
    const int nc = g.n_chunks;
    // surface roots
    DevBuf<int32_t> roots(g.S);
    LSPR_HIP(hipMemcpyAsync(roots.p, g.surf_root.data(), g.S * 4, hipMemcpyHostToDevice, s));
    ListParams lp{g.method == LSPR_DENSE ? 0.0 : g.theta, 1.0 / g.threshold, g.m2p_min_panels,
                  g.S, roots.p};
    DevBuf<int32_t> mc(nc), pc(nc);
    g.m2p_self.alloc(nc);
    g.p2p_self.alloc(nc);
    DevBuf<int64_t> pairs(2 * nc);
    const int64_t ntask = static_cast<int64_t>(nc) * g.S * SUBS;
    LSPR_REQUIRE(ntask < (1ll << 31), LSPR_E_INVALID, "too many list tasks");
    DevBuf<SubList> sub(ntask);
    DevBuf<SubPlace> place(ntask);
    const dim3 grid((ntask + 63) / 64), blk(64);
    hipLaunchKernelGGL(k_lists_count, grid, blk, 0, s, g.boxes.p, g.chunks.p, nc, lp, sub.p);
    hipLaunchKernelGGL(k_lists_place, dim3((nc + 63) / 64), dim3(64), 0, s, sub.p, nc, g.S,
                       place.p, mc.p, pc.p, g.m2p_self.p, g.p2p_self.p, pairs.p);
    LSPR_HIP(hipGetLastError());
    std::vector<int32_t> mh(nc), ph(nc);
    std::vector<int64_t> prh(2 * nc);
    g.m2p_self_h.resize(nc);
    g.p2p_self_h.resize(nc);
    Downloads down(s);
    down.add(mh.data(), mc.p, nc);
    down.add(ph.data(), pc.p, nc);
    down.add(prh.data(), pairs.p, 2 * nc);
    down.add(g.m2p_self_h.data(), g.m2p_self.p, nc);
    down.add(g.p2p_self_h.data(), g.p2p_self.p, nc);
    down.fetch();
    std::vector<int64_t> mo(nc + 1, 0), po(nc + 1, 0);
    g.p2p_pairs = 0;
    g.m2p_pairs = 0;
    for (int c = 0; c < nc; ++c) {
        mo[c + 1] = mo[c] + mh[c];
        po[c + 1] = po[c] + ph[c];
        g.p2p_pairs += prh[2 * c];
        g.m2p_pairs += prh[2 * c + 1];
    }
    g.n_m2p = mo[nc];
    g.n_p2p = po[nc];
    LSPR_REQUIRE(g.n_m2p < (1ll << 31) && g.n_p2p < (1ll << 31), LSPR_E_INVALID,
                 "interaction lists too long");
    g.m2p_off_h.resize(nc + 1);
    g.p2p_off_h.resize(nc + 1);
    for (int c = 0; c <= nc; ++c) {
        g.m2p_off_h[c] = static_cast<int32_t>(mo[c]);
        g.p2p_off_h[c] = static_cast<int32_t>(po[c]);
    }
    DevBuf<int64_t> mo_d(nc + 1), po_d(nc + 1);
    g.m2p_off.alloc(nc + 1);
    g.p2p_off.alloc(nc + 1);
    Uploads up(s);
    up.add(mo_d.p, mo.data(), nc + 1);
    up.add(po_d.p, po.data(), nc + 1);
    up.add(g.m2p_off.p, g.m2p_off_h.data(), nc + 1);
    up.add(g.p2p_off.p, g.p2p_off_h.data(), nc + 1);
    up.flush();
    g.m2p_box.alloc(std::max<int64_t>(g.n_m2p, 1));
    g.p2p_rng.alloc(std::max<int64_t>(g.n_p2p, 1));
    hipLaunchKernelGGL(k_lists_fill, grid, blk, 0, s, g.boxes.p, g.chunks.p, nc, lp, place.p,
                       mo_d.p, po_d.p, g.m2p_box.p, g.p2p_rng.p);
    LSPR_HIP(hipGetLastError());
    // the expansion boxes and direct ranges, for the tile and moment set-up
    g.m2p_box_h.resize(g.n_m2p);
    g.p2p_rng_h.resize(g.n_p2p);
    Downloads lists(s);
    lists.add(g.m2p_box_h.data(), g.m2p_box.p, g.m2p_box_h.size());
    lists.add(g.p2p_rng_h.data(), g.p2p_rng.p, g.p2p_rng_h.size());
    lists.fetch();
}

void build_near_table(Geometry& g) {
    hipStream_t s = g.stream;
    const int N = g.N;
    // one upload: surface roots, the fine rule and the Gauss-Legendre nodes of V_ii
    const std::vector<double> fine_h = rule_rows(g.Kf);
    std::vector<double> t, w;
    gauss_legendre(g.Nk, t, w);
    std::vector<int32_t> roots_h(g.surf_root.begin(), g.surf_root.end());
    roots_h.push_back(0);  // largest count
    DevBuf<int32_t> roots(g.S + 1);
    DevBuf<double> fine(fine_h.size()), t_d(t.size()), w_d(w.size());
    Uploads up(s);
    up.add(roots.p, roots_h.data(), g.S + 1);
    up.add(fine.p, fine_h.data(), fine_h.size());
    up.add(t_d.p, t.data(), t.size());
    up.add(w_d.p, w.data(), w.size());
    up.flush();
    NearParams np{1.0 / g.threshold, g.S, roots.p, roots.p + g.S};
    DevBuf<int64_t> cnt(N + 1);
    const dim3 grid((N + TPB - 1) / TPB), blk(TPB);
    // The counting walk keeps the first NEAR_CAP panels of each target; when no target has
    // more, they are moved into the table and the filling walk is not needed.
    constexpr int NEAR_CAP = 64;
    DevBuf<int32_t> slot;
    if (static_cast<size_t>(N) * NEAR_CAP * 4 <= (size_t(512) << 20)) slot.alloc(static_cast<size_t>(N) * NEAR_CAP);
    hipLaunchKernelGGL(k_near, grid, blk, 0, s, g.boxes.p, g.cen.p, g.area.p, N, np, false,
                       cnt.p, nullptr, nullptr, slot.p, NEAR_CAP);
    LSPR_HIP(hipGetLastError());
    scan_exclusive(cnt.p, cnt.p, N, s);
    int64_t nnz = 0;
    int32_t maxcnt = 0;  // largest count of a target
    LSPR_HIP(hipMemcpyAsync(&nnz, cnt.p + N, 8, hipMemcpyDeviceToHost, s));
    LSPR_HIP(hipMemcpyAsync(&maxcnt, np.maxcnt, 4, hipMemcpyDeviceToHost, s));
    LSPR_HIP(hipStreamSynchronize(s));
    LSPR_REQUIRE(nnz < (1ll << 31), LSPR_E_INVALID, "near-singular table too large");
    g.n_near = nnz;
    g.near_col.alloc(std::max<int64_t>(nnz, 1));
    g.near_dv.alloc(std::max<int64_t>(nnz, 1));
    g.near_dk.alloc(std::max<int64_t>(nnz, 1));
    if (slot.p != nullptr && maxcnt <= NEAR_CAP)
        hipLaunchKernelGGL(k_near_compact, dim3(N), dim3(64), 0, s, slot.p, NEAR_CAP, cnt.p,
                           g.near_col.p);
    else
        hipLaunchKernelGGL(k_near, grid, blk, 0, s, g.boxes.p, g.cen.p, g.area.p, N, np, true,
                           nullptr, cnt.p, g.near_col.p, nullptr, 0);
    LSPR_HIP(hipGetLastError());
    g.near_off64 = std::move(cnt);
    DevBuf<int32_t> row_of(std::max<int64_t>(nnz, 1));
    hipLaunchKernelGGL(k_row_of, grid, blk, 0, s, g.near_off64.p, N, row_of.p);
    LSPR_HIP(hipGetLastError());
    if (nnz > 0) {
        hipLaunchKernelGGL(k_near_values, dim3((nnz + TPB - 1) / TPB), dim3(TPB), 0, s, row_of.p,
                           g.near_col.p, nnz, g.tri.p, g.cen.p, g.nrm.p, g.area.p, g.far_rule.p,
                           g.K, fine.p, g.Kf, g.near_dv.p, g.near_dk.p);
        LSPR_HIP(hipGetLastError());
    }
    g.vself.alloc(N);
    hipLaunchKernelGGL(k_vself, grid, blk, 0, s, g.tri.p, g.cen.p, g.nrm.p, N, t_d.p, w_d.p,
                       g.Nk, g.vself.p);
    LSPR_HIP(hipGetLastError());
    LSPR_HIP(hipStreamSynchronize(s));
}

}  // namespace lspr
