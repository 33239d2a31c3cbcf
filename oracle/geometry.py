"""Panel geometry for the oracle (test infrastructure only).

Flat triangles with vertices counter-clockwise seen from outside (section "Boundary integral
expression of the dipole moment": normals point outwards); representative length
L = sqrt(2 * Area) (section "Integral evaluation").
"""
from __future__ import annotations

import numpy as np


def panel_geometry(verts: np.ndarray, tris: np.ndarray):
    """Area, unit outward normal, centroid and L = sqrt(2 A) of every panel."""
    v1 = verts[tris[:, 0]]
    v2 = verts[tris[:, 1]]
    v3 = verts[tris[:, 2]]
    cross = np.cross(v2 - v1, v3 - v1)
    twice_area = np.linalg.norm(cross, axis=1)
    area = 0.5 * twice_area
    normal = cross / twice_area[:, None]
    centroid = (v1 + v2 + v3) / 3.0
    return {"area": area, "normal": normal, "centroid": centroid, "L": np.sqrt(2.0 * area)}


def quadrature_nodes(verts: np.ndarray, tris: np.ndarray, bary: np.ndarray):
    """Physical quadrature nodes y[j, g] = sum_k bary[g, k] * v_k(j), shape [N, n_g, 3]."""
    corners = verts[tris]  # [N, 3 corners, 3 xyz]
    return np.einsum("gk,nkd->ngd", bary, corners)
