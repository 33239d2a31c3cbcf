"""Block linear systems and their solution for the oracle (test infrastructure only).

Unknowns per surface s (surface 0 is the metal sensor, s >= 1 the analytes): phi_s, the
scattered potential on the surface, and psi_s, its normal derivative on the interior side,
both constant per panel.  For a target panel i on surface t (Eqs. integral_eq_lspr and
integral_eq_lspr_system, written as matrices in Eqs. matrix_lspr and matrix_multi):

  interior row (own surface only):
      phi_i / 2 + sum_{j in t} K_ij phi_j - sum_{j in t} V_ij psi_j = 0
  exterior row (all surfaces):
      phi_i / 2 - sum_j K_ij phi_j + sum_j (eps_s(j) / eps_m) V_ij psi_j
          = sum_j ((eps_m - eps_s(j)) / eps_m) V_ij g_j,     g_j = dphi_inc/dn = -E . n_j

The incident potential of a uniform field E is phi_inc = -E . r.  Unknown order in the 2N
vector: all phi (panel order of the caller), then all psi; rows: all interior rows, then all
exterior rows.  Point charges q_k at r_k inside surface s (Eq. integral_eq_lspr_system, last row:
charges of an analyte) put (1 / (4 pi eps_s)) sum_k q_k / |x_i - r_k| on the right of the
interior rows of the panels i of surface s (eps_s relative, q_k divided by the vacuum
permittivity, in the units of the potential times length).
"""
from __future__ import annotations

import numpy as np

from .geometry import panel_geometry
from .operators import dense_operators
from .dipole import exterior_traces, dipole_moment, extinction_cross_section


def charge_potential(centroids, surf_id, charges, eps_surf):
    """Interior right-hand side of the point charges: for each panel i of surface s,
    (1 / (4 pi eps_s)) sum over the charges of surface s of q_k / |x_i - r_k|.  charges:
    (positions [Nq, 3], values [Nq], surfaces [Nq])."""
    pos, q, sq = (np.asarray(a) for a in charges)
    out = np.zeros(len(surf_id), dtype=np.complex128)
    for i in range(len(surf_id)):
        on = sq == surf_id[i]
        if np.any(on):
            r = np.linalg.norm(centroids[i][None, :] - pos[on], axis=1)
            out[i] = np.sum(q[on] / r) / (4.0 * np.pi * eps_surf[surf_id[i]])
    return out


def assemble_system(V, K, surf_id, normals, eps_m, eps_surf, e_field, centroids=None,
                    charges=None):
    """Dense complex matrix A [2N, 2N] and right-hand side b [2N] for one wavelength (with
    point charges: centroids [N, 3] and charges as in charge_potential)."""
    N = len(surf_id)
    same = surf_id[:, None] == surf_id[None, :]
    eps_panel = np.asarray(eps_surf)[surf_id]
    eye = np.eye(N)
    A = np.zeros((2 * N, 2 * N), dtype=np.complex128)
    A[:N, :N] = np.where(same, 0.5 * eye + K, 0.0)
    A[:N, N:] = np.where(same, -V, 0.0)
    A[N:, :N] = 0.5 * eye - K
    A[N:, N:] = V * (eps_panel / eps_m)[None, :]
    g = -(normals @ np.asarray(e_field, dtype=np.float64))
    b = np.zeros(2 * N, dtype=np.complex128)
    b[N:] = V @ (((eps_m - eps_panel) / eps_m) * g)
    if charges is not None and len(charges[1]) > 0:
        b[:N] = charge_potential(centroids, surf_id, charges, np.asarray(eps_surf))
    return A, b


def system_rows(V_rows, K_rows, rows, surf_id, eps_m, eps_surf):
    """Rows of A (Eq. matrix_multi) for the targets `rows`: interior rows [M, 2N] and exterior
    rows [M, 2N], from the same rows of V and K ([M, N] each).  The same entries as
    assemble_system, for targets of a mesh too large to assemble densely."""
    surf_id = np.asarray(surf_id)
    rows = np.asarray(rows)
    N = len(surf_id)
    M = len(rows)
    same = surf_id[rows][:, None] == surf_id[None, :]
    eps_panel = np.asarray(eps_surf)[surf_id]
    unit = np.zeros((M, N))
    unit[np.arange(M), rows] = 1.0
    interior = np.zeros((M, 2 * N), dtype=np.complex128)
    interior[:, :N] = np.where(same, 0.5 * unit + K_rows, 0.0)
    interior[:, N:] = np.where(same, -V_rows, 0.0)
    exterior = np.zeros((M, 2 * N), dtype=np.complex128)
    exterior[:, :N] = 0.5 * unit - K_rows
    exterior[:, N:] = V_rows * (eps_panel / eps_m)[None, :]
    return interior, exterior


def solve_lu(A, b):
    """Direct solve by LU with partial pivoting (LAPACK through numpy)."""
    return np.linalg.solve(A, b)


def gmres(matvec, b, tol=1e-10, restart=50, max_iter=2000):
    """Restarted GMRES(m) from x0 = 0, modified Gram-Schmidt Arnoldi, Givens rotations.

    Stops when ||b - A x||_2 / ||b||_2 <= tol (the Arnoldi estimate, checked against the true
    residual at every restart).  Returns (x, iterations, relative residual).
    """
    n = len(b)
    x = np.zeros(n, dtype=np.complex128)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    it = 0
    r = b.copy()
    beta = np.linalg.norm(r)
    while it < max_iter:
        m = min(restart, max_iter - it)
        Q = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        Q[0] = r / beta
        j_done = 0
        for j in range(m):
            w = matvec(Q[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(Q[i], w)
                w = w - H[i, j] * Q[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                Q[j + 1] = w / H[j + 1, j]
            # Givens rotation i acts on rows (i, i+1) as [x, y] -> [conj(c) x + conj(s) y,
            # -s x + c y]; rotation j is chosen so that it zeroes H[j+1, j].
            for i in range(j):
                hi, hn = H[i, j], H[i + 1, j]
                H[i, j] = np.conj(cs[i]) * hi + np.conj(sn[i]) * hn
                H[i + 1, j] = -sn[i] * hi + cs[i] * hn
            a, bb = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            cs[j], sn[j] = (a / den, bb / den) if den > 0 else (1.0, 0.0)
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            it += 1
            j_done = j + 1
            if abs(g[j + 1]) / bnorm <= tol:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + Q[:j_done].T @ y
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            break
    return x, it, float(np.linalg.norm(b - matvec(x)) / bnorm)


def solve(verts, tris, surf_id, lambdas, eps_medium, eps_surface, e_field, k_far=4, k_fine=19,
          n_k=9, threshold=0.5, method="lu", tol=1e-10, restart=50, max_iter=2000,
          charges=None):
    """Solve every wavelength densely; returns a dict of per-wavelength results.

    eps_medium [n_lambda] and eps_surface [n_lambda, n_surf] are complex relative
    permittivities; e_field is the real incident field vector.  `method` is "lu" or "gmres".
    charges: optional (positions, values, surfaces), see charge_potential.
    """
    surf_id = np.asarray(surf_id)
    geom = panel_geometry(verts, tris)
    V, K = dense_operators(verts, tris, k_far, k_fine, n_k, threshold)
    g = -(geom["normal"] @ np.asarray(e_field, dtype=np.float64))
    sensor = surf_id == 0
    N = len(tris)
    out = {k: [] for k in ("phi", "dphi", "p_sensor", "p_total", "cext_sensor", "cext_total",
                           "iters", "rel_resid")}
    for li, lam in enumerate(lambdas):
        em = complex(eps_medium[li])
        es = np.asarray(eps_surface[li], dtype=np.complex128)
        A, b = assemble_system(V, K, surf_id, geom["normal"], em, es, e_field,
                               geom["centroid"], charges)
        if method == "lu":
            x = solve_lu(A, b)
            iters, res = 0, float(np.linalg.norm(b - A @ x) / np.linalg.norm(b))
        else:
            x, iters, res = gmres(lambda v: A @ v, b, tol, restart, max_iter)
        phi, psi = x[:N], x[N:]
        phi_e, psi_e = exterior_traces(phi, psi, g, es[surf_id], em)
        q_s = dipole_moment(geom["area"], geom["normal"], geom["centroid"], phi_e, psi_e, sensor)
        q_t = dipole_moment(geom["area"], geom["normal"], geom["centroid"], phi_e, psi_e, None)
        out["phi"].append(phi)
        out["dphi"].append(psi)
        out["p_sensor"].append(em * q_s)
        out["p_total"].append(em * q_t)
        out["cext_sensor"].append(extinction_cross_section(q_s, e_field, lam, em))
        out["cext_total"].append(extinction_cross_section(q_t, e_field, lam, em))
        out["iters"].append(iters)
        out["rel_resid"].append(res)
    return {k: np.asarray(v) for k, v in out.items()}
