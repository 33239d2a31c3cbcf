// Cartesian Taylor expansion of the Laplace kernel used by the treecode (section
// "Acceleration strategies": Taylor expansions of order P, Duan & Krasny's treecode).
//
// For a source y near an expansion centre c and a target x,
//     1/|x - y| = sum_k F_k(c - x) (y - c)^k,   F_k = (1/k!) d^k/dy^k (1/|y - x|) at y = c,
// over multi-indices k = (kx, ky, kz), |k| <= P.  The coefficients obey (d = c - x)
//     |k| |d|^2 F_k + (2|k| - 1) sum_i d_i F_{k-e_i} + (|k| - 1) sum_i F_{k-2e_i} = 0,
// obtained from |y - x|^2 grad f = -(y - x) f by Euler's relation for the degree -1
// homogeneous f.  The double-layer kernel n.grad_y (1/|x-y|) expands with the same F_k and the
// moments sum w phi n.grad (y - c)^k.
//
// Because 1/|y - x| is harmonic, sum_i (m_i + 1)(m_i + 2) F_{m+2e_i} = 0 for every m, so every
// coefficient with kz >= 2 is a combination of coefficients of the same degree with smaller
// kz.  Folding the moments accordingly leaves (P + 1)^2 terms with kz in {0, 1} instead of
// (P+1)(P+2)(P+3)/6, without changing the sum; the recurrence above is closed on that subset.
#pragma once

#include <hip/hip_runtime.h>

namespace lspr {

template <int P>
struct Expansion {
    static constexpr int NF = (P + 1) * (P + 2) * (P + 3) / 6;  // full Cartesian terms
    static constexpr int NR = (P + 1) * (P + 1);                // folded terms (kz <= 1)
    static constexpr int NFOLD = NF - NR;                       // terms with kz >= 2

    // full terms, by increasing degree
    int fx[NF], fy[NF], fz[NF];
    // folded terms: indices into the full list, and recurrence predecessors within the folded
    // list (-1 where a component would be negative)
    int rfull[NR];
    int rx[NR], ry[NR], rz[NR], rn[NR];
    int m1[NR][3], m2[NR][3];
    // fold steps in order: full term src (kz >= 2) adds cx * M[src] to M[dx] and cy * M[src]
    // to M[dy]
    int fsrc[NFOLD > 0 ? NFOLD : 1], fdx[NFOLD > 0 ? NFOLD : 1], fdy[NFOLD > 0 ? NFOLD : 1];
    double fcx[NFOLD > 0 ? NFOLD : 1], fcy[NFOLD > 0 ? NFOLD : 1];

    constexpr int full_index(int x, int y, int z) const {
        for (int t = 0; t < NF; ++t)
            if (fx[t] == x && fy[t] == y && fz[t] == z) return t;
        return -1;
    }
    constexpr int red_index(int x, int y, int z) const {
        if (x < 0 || y < 0 || z < 0 || z > 1) return -1;
        for (int t = 0; t < NR; ++t)
            if (rx[t] == x && ry[t] == y && rz[t] == z) return t;
        return -1;
    }

    constexpr Expansion() : fx(), fy(), fz(), rfull(), rx(), ry(), rz(), rn(), m1(), m2(),
                            fsrc(), fdx(), fdy(), fcx(), fcy() {
        int t = 0;
        for (int n = 0; n <= P; ++n)
            for (int x = n; x >= 0; --x)
                for (int y = n - x; y >= 0; --y) {
                    fx[t] = x;
                    fy[t] = y;
                    fz[t] = n - x - y;
                    ++t;
                }
        int r = 0;
        for (int n = 0; n <= P; ++n)
            for (int z = 0; z <= 1 && z <= n; ++z)
                for (int x = n - z; x >= 0; --x) {
                    rx[r] = x;
                    ry[r] = n - z - x;
                    rz[r] = z;
                    rn[r] = n;
                    ++r;
                }
        for (int q = 0; q < NR; ++q) {
            rfull[q] = full_index(rx[q], ry[q], rz[q]);
            m1[q][0] = red_index(rx[q] - 1, ry[q], rz[q]);
            m1[q][1] = red_index(rx[q], ry[q] - 1, rz[q]);
            m1[q][2] = red_index(rx[q], ry[q], rz[q] - 1);
            m2[q][0] = red_index(rx[q] - 2, ry[q], rz[q]);
            m2[q][1] = red_index(rx[q], ry[q] - 2, rz[q]);
            m2[q][2] = red_index(rx[q], ry[q], rz[q] - 2);
        }
        int f = 0;
        for (int z = P; z >= 2; --z)
            for (int n = z; n <= P; ++n)
                for (int x = n - z; x >= 0; --x) {
                    const int y = n - z - x;
                    // k = (x, y, z) = m + 2 e_z with m = (x, y, z - 2)
                    const double den = double(z - 1) * double(z);
                    fsrc[f] = full_index(x, y, z);
                    fdx[f] = full_index(x + 2, y, z - 2);
                    fdy[f] = full_index(x, y + 2, z - 2);
                    fcx[f] = -double(x + 1) * double(x + 2) / den;
                    fcy[f] = -double(y + 1) * double(y + 2) / den;
                    ++f;
                }
    }
};

// Taylor coefficients F (folded terms) for d = c - x, without any 1/(4 pi).
template <class T, int P>
__device__ __forceinline__ void taylor_coefficients(T dx, T dy, T dz, T* F) {
    constexpr Expansion<P> E{};
    const T r2 = dx * dx + dy * dy + dz * dz;
    const T inv_r2 = T(1) / r2;
    F[0] = T(1) / sqrt(r2);
#pragma unroll
    for (int q = 1; q < Expansion<P>::NR; ++q) {
        const int n = E.rn[q];
        T s1 = T(0), s2 = T(0);
        if (E.m1[q][0] >= 0) s1 += dx * F[E.m1[q][0]];
        if (E.m1[q][1] >= 0) s1 += dy * F[E.m1[q][1]];
        if (E.m1[q][2] >= 0) s1 += dz * F[E.m1[q][2]];
        if (E.m2[q][0] >= 0) s2 += F[E.m2[q][0]];
        if (E.m2[q][1] >= 0) s2 += F[E.m2[q][1]];
        if (E.m2[q][2] >= 0) s2 += F[E.m2[q][2]];
        F[q] = -(T(2 * n - 1) * s1 + T(n - 1) * s2) * inv_r2 * T(1.0 / n);
    }
}

}  // namespace lspr
