// Post-processing: exterior traces, dipole moment and reordering (section "Boundary integral
// expression of the dipole moment"; Eqs. electrostatic_scatter and cext_fwa).
//
// Exterior traces from the interface condition: phi_out = phi and
//     psi_out = r_s psi - (1 - r_s) g,   r_s = eps_s / eps_m,  g = dphi_inc/dn = -E . n.
// Dipole moment.  Green's second identity for phi_out and the coordinate x_k over the exterior
// region, closed by a large sphere on which phi_out ~ p . r_hat / (4 pi eps_m r^2), gives with
// outward normals q = p / eps_m = surface integral of (phi_out n - x psi_out); the printed
// Eq. dipole_def_gauss_i_final has the opposite overall sign, which would make the sphere's
// cross-section negative.  With constant values on a flat panel the integral of x over the
// panel is Area * centroid.  C_ext follows on the host from q.
#include "system.hpp"

namespace lspr {

namespace {

constexpr int DT = 256;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Per block partial sums of q_sensor (3 complex) and q_total (3 complex): part[col][blk][12].
__global__ void __launch_bounds__(DT) k_dipole(const double2* __restrict__ x, int N,
                                               const double2* __restrict__ ratio, int S,
                                               const int32_t* __restrict__ surf,
                                               const double* __restrict__ area,
                                               const double* __restrict__ nrm,
                                               const double* __restrict__ cen, double e0,
                                               double e1, double e2, double* __restrict__ part,
                                               int nblk) {
    __shared__ double red[12][DT];
    const int col = blockIdx.y;
    const double2* xc = x + static_cast<int64_t>(col) * 2 * N;
    double acc[12];
    for (int k = 0; k < 12; ++k) acc[k] = 0.0;
    for (int i = blockIdx.x * DT + threadIdx.x; i < N; i += nblk * DT) {
        const double2 phi = xc[i], psi = xc[N + i];
        const double2 r = ratio[col * S + surf[i]];
        const double* n = nrm + 3 * i;
        const double* c = cen + 3 * i;
        const double gi = -(e0 * n[0] + e1 * n[1] + e2 * n[2]);
        const double2 rp = cmul(r, psi);
        const double2 po = make_double2(rp.x - (1.0 - r.x) * gi, rp.y + r.y * gi);
        const double A = area[i];
        const bool sensor = surf[i] == 0;
        for (int d = 0; d < 3; ++d) {
            const double vr = A * (phi.x * n[d] - c[d] * po.x);
            const double vi = A * (phi.y * n[d] - c[d] * po.y);
            acc[6 + 2 * d] += vr;
            acc[7 + 2 * d] += vi;
            if (sensor) {
                acc[2 * d] += vr;
                acc[2 * d + 1] += vi;
            }
        }
    }
    for (int k = 0; k < 12; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int off = DT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int k = 0; k < 12; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x < 12)
        part[(static_cast<int64_t>(col) * nblk + blockIdx.x) * 12 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_unpermute(const double2* __restrict__ x, int N, int B,
                            const int32_t* __restrict__ perm, double2* __restrict__ phi,
                            double2* __restrict__ dphi) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(N) * B) return;
    const int b = static_cast<int>(t / N), i = static_cast<int>(t % N);
    const int o = perm[i];
    if (phi) phi[static_cast<int64_t>(b) * N + o] = x[static_cast<int64_t>(b) * 2 * N + i];
    if (dphi) dphi[static_cast<int64_t>(b) * N + o] = x[static_cast<int64_t>(b) * 2 * N + N + i];
}

// dir 0: out (sorted) <- in (caller order); dir 1: out (caller order) <- in (sorted)
__global__ void k_reorder(const double2* __restrict__ in, double2* __restrict__ out, int N, int B,
                          const int32_t* __restrict__ perm, int dir) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= static_cast<int64_t>(N) * B) return;
    const int b = static_cast<int>(t / N), i = static_cast<int>(t % N);
    const int o = perm[i];
    const int64_t base = static_cast<int64_t>(b) * 2 * N;
    if (dir == 0) {
        out[base + i] = in[base + o];
        out[base + N + i] = in[base + N + o];
    } else {
        out[base + o] = in[base + i];
        out[base + N + o] = in[base + N + i];
    }
}

}  // namespace

void dipole_moments(Geometry& g, int B, const double2* ratio_d, const double* e_field,
                    const double2* x, std::vector<double>& q, hipStream_t s) {
    const int nblk = std::min(256, (g.N + DT - 1) / DT);
    DevBuf<double> part(static_cast<size_t>(B) * nblk * 12);
    hipLaunchKernelGGL(k_dipole, dim3(nblk, B), dim3(DT), 0, s, x, g.N, ratio_d, g.S, g.surf.p,
                       g.area.p, g.nrm.p, g.cen.p, e_field[0], e_field[1], e_field[2], part.p,
                       nblk);
    LSPR_HIP(hipGetLastError());
    std::vector<double> h(part.n);
    LSPR_HIP(hipMemcpyAsync(h.data(), part.p, h.size() * 8, hipMemcpyDeviceToHost, s));
    LSPR_HIP(hipStreamSynchronize(s));
    q.assign(static_cast<size_t>(B) * 12, 0.0);
    for (int b = 0; b < B; ++b)
        for (int k = 0; k < nblk; ++k)
            for (int e = 0; e < 12; ++e) q[b * 12 + e] += h[(static_cast<size_t>(b) * nblk + k) * 12 + e];
}

void unpermute(Geometry& g, int B, const double2* x, double2* phi, double2* dphi, hipStream_t s) {
    const int64_t t = static_cast<int64_t>(g.N) * B;
    hipLaunchKernelGGL(k_unpermute, dim3((t + 255) / 256), dim3(256), 0, s, x, g.N, B, g.perm.p,
                       phi, dphi);
    LSPR_HIP(hipGetLastError());
}

void to_sorted(Geometry& g, int B, const double2* in, double2* out, hipStream_t s) {
    const int64_t t = static_cast<int64_t>(g.N) * B;
    hipLaunchKernelGGL(k_reorder, dim3((t + 255) / 256), dim3(256), 0, s, in, out, g.N, B,
                       g.perm.p, 0);
    LSPR_HIP(hipGetLastError());
}

void from_sorted(Geometry& g, int B, const double2* in, double2* out, hipStream_t s) {
    const int64_t t = static_cast<int64_t>(g.N) * B;
    hipLaunchKernelGGL(k_reorder, dim3((t + 255) / 256), dim3(256), 0, s, in, out, g.N, B,
                       g.perm.p, 1);
    LSPR_HIP(hipGetLastError());
}

}  // namespace lspr
