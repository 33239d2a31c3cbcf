// Right block-Jacobi preconditioner with the 2x2 self-panel block of panel i (K_ii = 0 on a flat
// panel): M [phi; psi] = [phi / 2 - V_ii psi; phi / 2 + r V_ii psi] for the row pair of
// Eq. matrix_lspr, r = eps_s / eps_m.  Its inverse applied to (a, b):
//     phi = 2 (r a + b) / (1 + r),   psi = (b - a) / (V_ii (1 + r)).
#pragma once

#include <hip/hip_runtime.h>

namespace lspr {

// vii: the singular self-integral V_ii (already divided by 4 pi)
__device__ __forceinline__ void block_jacobi(double2 a, double2 b, double2 r, double vii,
                                             double2& phi, double2& psi) {
    const double2 onep = make_double2(1.0 + r.x, r.y);
    const double2 ra = make_double2(r.x * a.x - r.y * a.y, r.x * a.y + r.y * a.x);
    const double2 u = make_double2(2.0 * (ra.x + b.x), 2.0 * (ra.y + b.y));
    const double2 v = make_double2((b.x - a.x) / vii, (b.y - a.y) / vii);
    const double d = onep.x * onep.x + onep.y * onep.y;
    phi = make_double2((u.x * onep.x + u.y * onep.y) / d, (u.y * onep.x - u.x * onep.y) / d);
    psi = make_double2((v.x * onep.x + v.y * onep.y) / d, (v.y * onep.x - v.x * onep.y) / d);
}

}  // namespace lspr
