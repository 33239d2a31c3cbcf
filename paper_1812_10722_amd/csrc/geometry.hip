// Panel geometry and Morton ordering (set-up, once per mesh).
//
// Flat triangles, counter-clockwise seen from outside; area A, unit outward normal n,
// centroid c (the collocation point) and representative length L = sqrt(2 A) (sections
// "Discretization and linear system" and "Integral evaluation").  Panels are reordered by the
// Morton code of their centroid inside one bounding cube shared by all surfaces, surface by
// surface, so that octree boxes and target groups are contiguous index ranges (section
// "Acceleration strategies": sources grouped geometrically in the boxes of an octree).
#include <cfloat>
#include <cmath>

#include "primitives.hpp"

namespace lspr {

namespace {

constexpr int TPB = 256;

// Copy one surface's triangles into the per-panel vertex array (caller's order) and flag bad
// indices or degenerate panels.
__global__ void k_gather(const double* __restrict__ vert, int n_vert,
                         const int32_t* __restrict__ tri, int n_tri, int offset, int surf_id,
                         double* __restrict__ tri_out, int32_t* __restrict__ surf_out,
                         int* __restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_tri) return;
    double v[9];
    for (int k = 0; k < 3; ++k) {
        const int vi = tri[3 * i + k];
        if (vi < 0 || vi >= n_vert) {
            atomicOr(bad, 1);
            for (int d = 0; d < 3; ++d) v[3 * k + d] = 0.0;
        } else {
            for (int d = 0; d < 3; ++d) v[3 * k + d] = vert[3 * vi + d];
        }
    }
    const double ax = v[3] - v[0], ay = v[4] - v[1], az = v[5] - v[2];
    const double bx = v[6] - v[0], by = v[7] - v[1], bz = v[8] - v[2];
    const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
    const double cn = sqrt(cx * cx + cy * cy + cz * cz);
    const double scale = fmax(fmax(ax * ax + ay * ay + az * az, bx * bx + by * by + bz * bz), 1e-300);
    if (!(cn > 1e-14 * scale)) atomicOr(bad, 2);
    for (int k = 0; k < 9; ++k) tri_out[9 * (offset + i) + k] = v[k];
    surf_out[offset + i] = surf_id;
}

// Bounding box of all vertices: per-block min/max, then a second pass on the host.
__global__ void k_bbox(const double* __restrict__ tri, int n, double* __restrict__ part) {
    __shared__ double s[6][TPB];
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        for (int k = 0; k < 3; ++k)
            for (int d = 0; d < 3; ++d) {
                const double x = tri[9 * i + 3 * k + d];
                lo[d] = fmin(lo[d], x);
                hi[d] = fmax(hi[d], x);
            }
    }
    for (int d = 0; d < 3; ++d) {
        s[d][threadIdx.x] = lo[d];
        s[3 + d][threadIdx.x] = hi[d];
    }
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int d = 0; d < 3; ++d) {
                s[d][threadIdx.x] = fmin(s[d][threadIdx.x], s[d][threadIdx.x + off]);
                s[3 + d][threadIdx.x] = fmax(s[3 + d][threadIdx.x], s[3 + d][threadIdx.x + off]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 6; ++d) part[6 * blockIdx.x + d] = s[d][0];
}

__device__ inline uint64_t spread3(uint64_t x) {  // 16 bits -> every third bit of 48
    x &= 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

// key = surface id above a 48-bit Morton code of the centroid (16 bits per axis).
__global__ void k_morton(const double* __restrict__ tri, const int32_t* __restrict__ surf,
                         int n, double ox, double oy, double oz, double half,
                         uint64_t* __restrict__ keys, int32_t* __restrict__ idx) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double* v = tri + 9 * i;
    const double c[3] = {(v[0] + v[3] + v[6]) / 3.0, (v[1] + v[4] + v[7]) / 3.0,
                         (v[2] + v[5] + v[8]) / 3.0};
    const double o[3] = {ox, oy, oz};
    uint64_t q[3];
    for (int d = 0; d < 3; ++d) {
        double u = (c[d] - (o[d] - half)) / (2.0 * half) * 65536.0;
        u = fmin(fmax(u, 0.0), 65535.0);
        q[d] = static_cast<uint64_t>(u);
    }
    keys[i] = (static_cast<uint64_t>(surf[i]) << 48) |
              (spread3(q[0]) << 2) | (spread3(q[1]) << 1) | spread3(q[2]);
    idx[i] = i;
}

// Sorted per-panel geometry and the far-field source record of precision T:
//   rec[0..3] = (n_x, n_y, n_z, A),  rec[4+4g .. 7+4g] = (y_g - c, w_g) for node g,
// with w_g = A * omega_g of the far rule.
template <class T>
__global__ void k_permute(const double* __restrict__ tri_in, const int32_t* __restrict__ surf_in,
                          const int32_t* __restrict__ perm, int n, const double* __restrict__ rule,
                          int K, double* __restrict__ tri, double* __restrict__ cen,
                          double* __restrict__ nrm, double* __restrict__ area,
                          int32_t* __restrict__ surf, int32_t* __restrict__ iperm,
                          T* __restrict__ rec) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int src = perm[i];
    double v[9];
    for (int k = 0; k < 9; ++k) {
        v[k] = tri_in[9 * src + k];
        tri[9 * i + k] = v[k];
    }
    surf[i] = surf_in[src];
    iperm[src] = i;
    const double ax = v[3] - v[0], ay = v[4] - v[1], az = v[5] - v[2];
    const double bx = v[6] - v[0], by = v[7] - v[1], bz = v[8] - v[2];
    const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
    const double twice = sqrt(cx * cx + cy * cy + cz * cz);
    const double A = 0.5 * twice;
    const double n3[3] = {cx / twice, cy / twice, cz / twice};
    const double c3[3] = {(v[0] + v[3] + v[6]) / 3.0, (v[1] + v[4] + v[7]) / 3.0,
                          (v[2] + v[5] + v[8]) / 3.0};
    for (int d = 0; d < 3; ++d) {
        cen[3 * i + d] = c3[d];
        nrm[3 * i + d] = n3[d];
    }
    area[i] = A;
    T* r = rec + static_cast<size_t>(i) * (4 + 4 * K);
    r[0] = static_cast<T>(n3[0]);
    r[1] = static_cast<T>(n3[1]);
    r[2] = static_cast<T>(n3[2]);
    r[3] = static_cast<T>(A);
    for (int g = 0; g < K; ++g) {
        const double b0 = rule[4 * g], b1 = rule[4 * g + 1], b2 = rule[4 * g + 2];
        for (int d = 0; d < 3; ++d) {
            const double y = b0 * v[d] + b1 * v[3 + d] + b2 * v[6 + d];
            r[4 + 4 * g + d] = static_cast<T>(y - c3[d]);
        }
        r[4 + 4 * g + 3] = static_cast<T>(A * rule[4 * g + 3]);
    }
}

}  // namespace

void build_geometry(Geometry& g, const lspr_surface* surfaces, int n_surf) {
    hipStream_t s = g.stream;
    g.S = n_surf;
    int N = 0;
    std::vector<int> offs(n_surf + 1, 0);
    for (int k = 0; k < n_surf; ++k) {
        offs[k] = N;
        N += surfaces[k].n_tri;
    }
    offs[n_surf] = N;
    g.N = N;
    DevBuf<double> tri_in(static_cast<size_t>(N) * 9);
    DevBuf<int32_t> surf_in(N);
    DevBuf<int> bad(1);
    LSPR_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), s));
    for (int k = 0; k < n_surf; ++k) {
        const int n = surfaces[k].n_tri;
        hipLaunchKernelGGL(k_gather, dim3((n + TPB - 1) / TPB), dim3(TPB), 0, s,
                           surfaces[k].vert, surfaces[k].n_vert, surfaces[k].tri, n, offs[k], k,
                           tri_in.p, surf_in.p, bad.p);
        LSPR_HIP(hipGetLastError());
    }
    int bad_h = 0;
    LSPR_HIP(hipMemcpyAsync(&bad_h, bad.p, sizeof(int), hipMemcpyDeviceToHost, s));
    // bounding cube
    const int nb = std::min(256, (N + TPB - 1) / TPB);
    DevBuf<double> part(6 * nb);
    hipLaunchKernelGGL(k_bbox, dim3(nb), dim3(TPB), 0, s, tri_in.p, N, part.p);
    LSPR_HIP(hipGetLastError());
    std::vector<double> ph(6 * nb);
    LSPR_HIP(hipMemcpyAsync(ph.data(), part.p, ph.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    LSPR_HIP(hipStreamSynchronize(s));
    LSPR_REQUIRE(!(bad_h & 1), LSPR_E_MESH, "triangle vertex index out of range");
    LSPR_REQUIRE(!(bad_h & 2), LSPR_E_MESH, "degenerate (zero-area) panel");
    double lo[3] = {DBL_MAX, DBL_MAX, DBL_MAX}, hi[3] = {-DBL_MAX, -DBL_MAX, -DBL_MAX};
    for (int b = 0; b < nb; ++b)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], ph[6 * b + d]);
            hi[d] = std::max(hi[d], ph[6 * b + 3 + d]);
        }
    double half = 0.0;
    for (int d = 0; d < 3; ++d) {
        g.origin[d] = 0.5 * (lo[d] + hi[d]);
        half = std::max(half, 0.5 * (hi[d] - lo[d]));
    }
    g.half = half * (1.0 + 1e-9) + 1e-12;

    // Morton order (surface id in the high bits keeps surfaces contiguous)
    DevBuf<uint64_t> keys(N);
    g.perm.alloc(N);
    hipLaunchKernelGGL(k_morton, dim3((N + TPB - 1) / TPB), dim3(TPB), 0, s, tri_in.p, surf_in.p,
                       N, g.origin[0], g.origin[1], g.origin[2], g.half, keys.p, g.perm.p);
    LSPR_HIP(hipGetLastError());
    int sbits = 0;
    while ((1 << sbits) < n_surf) ++sbits;
    radix_sort_pairs(keys.p, g.perm.p, N, 48 + sbits, s);
    g.morton = std::move(keys);

    // far rule as (b0, b1, b2, w) rows
    std::vector<double> bary, w;
    LSPR_REQUIRE(triangle_rule(g.K, bary, w), LSPR_E_INVALID, "unsupported k_far");
    std::vector<double> rule(4 * g.K);
    for (int q = 0; q < g.K; ++q) {
        rule[4 * q] = bary[3 * q];
        rule[4 * q + 1] = bary[3 * q + 1];
        rule[4 * q + 2] = bary[3 * q + 2];
        rule[4 * q + 3] = w[q];
    }
    DevBuf<double> rule_d(rule.size());
    LSPR_HIP(hipMemcpyAsync(rule_d.p, rule.data(), rule.size() * sizeof(double),
                            hipMemcpyHostToDevice, s));
    g.tri.alloc(static_cast<size_t>(N) * 9);
    g.cen.alloc(static_cast<size_t>(N) * 3);
    g.nrm.alloc(static_cast<size_t>(N) * 3);
    g.area.alloc(N);
    g.surf.alloc(N);
    g.iperm.alloc(N);
    const size_t rs = static_cast<size_t>(N) * (4 + 4 * g.K);
    if (g.need32) {
        g.src32.alloc(rs);
        hipLaunchKernelGGL(k_permute<float>, dim3((N + TPB - 1) / TPB), dim3(TPB), 0, s,
                           tri_in.p, surf_in.p, g.perm.p, N, rule_d.p, g.K, g.tri.p, g.cen.p,
                           g.nrm.p, g.area.p, g.surf.p, g.iperm.p, g.src32.p);
        LSPR_HIP(hipGetLastError());
    }
    if (g.need64) {
        g.src64.alloc(rs);
        hipLaunchKernelGGL(k_permute<double>, dim3((N + TPB - 1) / TPB), dim3(TPB), 0, s,
                           tri_in.p, surf_in.p, g.perm.p, N, rule_d.p, g.K, g.tri.p, g.cen.p,
                           g.nrm.p, g.area.p, g.surf.p, g.iperm.p, g.src64.p);
    }
    LSPR_HIP(hipGetLastError());
    g.surf_start = offs;
    LSPR_HIP(hipStreamSynchronize(s));
}

}  // namespace lspr
