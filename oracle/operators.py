"""Dense Laplace single- and double-layer matrices for the oracle (test infrastructure only).

Matrix entries (Eq. layers_element, collocation at panel centroids x_i):

    V_ij = integral over panel j of G(x_i, y) dA_y,
    K_ij = integral over panel j of dG/dn_y (x_i, y) dA_y = n_j . (x_i - y) / (4 pi |x_i - y|^3),
    G(x, y) = 1 / (4 pi |x - y|).

The normal derivative is taken at the source point with the outward normal (Eq. double_layer);
with that convention the interior identity phi/2 + K phi - V dphi/dn = 0 holds for phi = 1, so
K applied to a constant is -1/2 on a closed surface.

Integration regions (section "Integral evaluation"):
  * singular (i == j): K_ii = 0 because x_i lies in the flat panel's plane; V_ii by the
    semi-analytic scheme with N_k Gauss-Legendre nodes on each edge;
  * near-singular (i != j and |x_i - c_j| <= L_j / threshold, threshold 0.5 giving the
    paper's "2L or less"): the K_fine-point rule;
  * far: the K-point rule.
"""
from __future__ import annotations

import numpy as np

from .geometry import panel_geometry, quadrature_nodes
from .quadrature import triangle_rule, gauss_legendre

FOUR_PI = 4.0 * np.pi


def singular_v_semianalytic(tri: np.ndarray, x: np.ndarray, n_k: int) -> float:
    """V of a flat panel at a point x inside it (section "Integral evaluation", singular case).

    Polar coordinates about x split the panel into three sub-triangles (x, edge).  For an edge
    whose line lies at perpendicular distance h from x, the ray at angle alpha (measured from
    the perpendicular) meets the edge at radius h / cos(alpha), and the radial integral of
    (1/rho) rho drho is that radius exactly.  The remaining integral over alpha, between the
    angles of the edge's end points, takes n_k Gauss-Legendre nodes, i.e. n_k points on the
    edge.
    """
    t, w = gauss_legendre(n_k)
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    n = n / np.linalg.norm(n)
    total = 0.0
    for e in range(3):
        a, b = tri[e], tri[(e + 1) % 3]
        edge = b - a
        length = np.linalg.norm(edge)
        u = edge / length
        h = np.dot(a - x, np.cross(edge, n) / length)  # > 0 for x inside the panel
        alpha_a = np.arctan2(np.dot(a - x, u), h)
        alpha_b = np.arctan2(np.dot(b - x, u), h)
        half = 0.5 * (alpha_b - alpha_a)
        alpha = 0.5 * (alpha_b + alpha_a) + half * t
        total += np.sum(half * w * h / np.cos(alpha))
    return total / FOUR_PI


def singular_v_closed_form(tri: np.ndarray, x: np.ndarray) -> float:
    """Exact V of a flat panel at an interior point: (1/4pi) sum_edges h [asinh(s)]_{s_a}^{s_b}."""
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    n = n / np.linalg.norm(n)
    total = 0.0
    for e in range(3):
        a, b = tri[e], tri[(e + 1) % 3]
        edge = b - a
        length = np.linalg.norm(edge)
        u = edge / length
        h = np.dot(a - x, np.cross(edge, n) / length)
        sa, sb = np.dot(a - x, u), np.dot(b - x, u)
        total += h * (np.arcsinh(sb / h) - np.arcsinh(sa / h))
    return total / FOUR_PI


def near_singular_mask(centroids_t: np.ndarray, rows: np.ndarray, centroids: np.ndarray,
                       L: np.ndarray, threshold: float) -> np.ndarray:
    """[M, N] mask of near-singular pairs: |x_i - c_j| <= L_j / threshold and i != j."""
    d = np.linalg.norm(centroids_t[:, None, :] - centroids[None, :, :], axis=2)
    mask = d <= (L / threshold)[None, :]
    mask[np.arange(len(rows)), rows] = False
    return mask


def _rule_sums(x: np.ndarray, nodes: np.ndarray, weights: np.ndarray, normals: np.ndarray):
    """sum_g w_g G(x, y_g) and sum_g w_g dG/dn_y(x, y_g) for targets x [M,3] vs panels.

    nodes [..., n_g, 3], weights [..., n_g] (already multiplied by the panel area) and normals
    [..., 3] broadcast against x: x of shape [P, 1, 3] pairs targets and panels one to one,
    x of shape [M, 1, 1, 3] against nodes [1, N, n_g, 3] gives all M x N pairs.
    """
    d = x - nodes
    r = np.linalg.norm(d, axis=-1)
    v = np.sum(weights / r, axis=-1) / FOUR_PI
    dn = np.einsum("...gd,...d->...g", d, normals)
    k = np.sum(weights * dn / r ** 3, axis=-1) / FOUR_PI
    return v, k


def operator_rows(verts, tris, rows=None, k_far=4, k_fine=19, n_k=9, threshold=0.5,
                  block_bytes=256 << 20):
    """Rows `rows` (default all) of the dense V and K matrices, FP64, shape [M, N] each."""
    geom = panel_geometry(verts, tris)
    N = len(tris)
    rows = np.arange(N) if rows is None else np.asarray(rows)
    M = len(rows)
    bf, wf = triangle_rule(k_far)
    bn, wn = triangle_rule(k_fine)
    nodes_f = quadrature_nodes(verts, tris, bf)                 # [N, K, 3]
    wts_f = geom["area"][:, None] * wf[None, :]                 # [N, K]
    nodes_n = quadrature_nodes(verts, tris, bn)                 # [N, K_fine, 3]
    wts_n = geom["area"][:, None] * wn[None, :]
    x = geom["centroid"][rows]
    V = np.empty((M, N))
    K = np.empty((M, N))
    blk = max(1, int(block_bytes // (N * k_far * 3 * 8 * 4)))
    for s in range(0, M, blk):
        e = min(M, s + blk)
        xb = x[s:e]
        rb = rows[s:e]
        with np.errstate(divide="ignore", invalid="ignore"):
            v, k = _rule_sums(xb[:, None, None, :], nodes_f[None], wts_f[None],
                              geom["normal"][None])
        # near-singular pairs: replace the far rule by the fine rule
        near = near_singular_mask(xb, rb, geom["centroid"], geom["L"], threshold)
        bi, bj = np.nonzero(near)
        if len(bi):
            vn, kn = _rule_sums(xb[bi][:, None, :], nodes_n[bj], wts_n[bj], geom["normal"][bj])
            v[bi, bj] = vn
            k[bi, bj] = kn
        # singular pairs: semi-analytic V, K = 0 on a flat panel
        for local, i in enumerate(rb):
            v[local, i] = singular_v_semianalytic(verts[tris[i]], geom["centroid"][i], n_k)
            k[local, i] = 0.0
        V[s:e] = v
        K[s:e] = k
    return V, K


def dense_operators(verts, tris, k_far=4, k_fine=19, n_k=9, threshold=0.5):
    """Full dense V and K ([N, N] FP64 each)."""
    return operator_rows(verts, tris, None, k_far, k_fine, n_k, threshold)
