"""Seeded synthetic surface meshes: octahedral geodesic spheres and perturbed ellipsoids.

These generators produce input data only (vertex and triangle arrays); they hold none of the
boundary-element arithmetic.  Both the oracle tests and the HIP path receive the same arrays.

Conventions (the paper's discretisation, section "Discretization and linear system"): flat
triangles, vertex order counter-clockwise seen from outside so that the right-hand normal
(v2 - v1) x (v3 - v1) points out of the enclosed region.  Lengths are in nm.
"""
from __future__ import annotations

import numpy as np

# Octahedron corner directions per octant sign pattern.
_OCTANTS = [(sx, sy, sz) for sx in (1, -1) for sy in (1, -1) for sz in (1, -1)]


def octahedral_grid(nu: int):
    """Subdivided octahedron with 8*nu**2 faces, vertices on the octahedron |x|+|y|+|z| = 1.

    Returns (verts float64 [n_v,3], tris int32 [8 nu^2, 3]), counter-clockwise from outside.
    Shared edge vertices are merged by their exact integer lattice coordinates.
    """
    if nu < 1:
        raise ValueError("nu must be >= 1")
    index = {}
    verts = []
    tris = []

    def vid(key):
        v = index.get(key)
        if v is None:
            v = len(verts)
            index[key] = v
            verts.append(key)
        return v

    for sx, sy, sz in _OCTANTS:
        a = np.array([sx, 0, 0])
        b = np.array([0, sy, 0])
        c = np.array([0, 0, sz])
        if sx * sy * sz < 0:  # keep the face counter-clockwise seen from outside
            b, c = c, b

        def lat(i, j):
            # nu times the grid point a + (b - a) i/nu + (c - a) j/nu: an exact integer key
            q = a * (nu - i - j) + b * i + c * j
            return (int(q[0]), int(q[1]), int(q[2]))

        for i in range(nu):
            for j in range(nu - i):
                v0 = vid(lat(i, j))
                v1 = vid(lat(i + 1, j))
                v2 = vid(lat(i, j + 1))
                tris.append((v0, v1, v2))
                if i + j < nu - 1:
                    v3 = vid(lat(i + 1, j + 1))
                    tris.append((v1, v3, v2))
    verts = np.asarray(verts, dtype=np.float64) / nu
    return verts, np.asarray(tris, dtype=np.int32)


def octasphere(nu: int, radius: float = 1.0, center=(0.0, 0.0, 0.0)):
    """Octahedral geodesic sphere: 8*nu**2 flat triangles, vertices projected onto the sphere."""
    v, t = octahedral_grid(nu)
    v = v / np.linalg.norm(v, axis=1, keepdims=True) * radius
    return v + np.asarray(center, dtype=np.float64), t


def graded_octasphere(nu: int, radius: float = 1.0, strength: float = 0.6):
    """Sphere with a deliberately non-uniform panel size (finer towards +z).

    Vertices of the octasphere are moved along meridians by the polar-angle map
    theta -> theta - (strength/2) sin(theta), which is monotone for strength < 2 and fixes both
    poles; panel areas then vary by a factor of several across the surface.  Used by tests
    that must tell V_ij from V_ji.
    """
    v, t = octahedral_grid(nu)
    v = v / np.linalg.norm(v, axis=1, keepdims=True)
    theta = np.arccos(np.clip(v[:, 2], -1.0, 1.0))
    phi = np.arctan2(v[:, 1], v[:, 0])
    theta2 = theta - strength * np.sin(theta) * 0.5
    out = np.stack([np.sin(theta2) * np.cos(phi), np.sin(theta2) * np.sin(phi), np.cos(theta2)], 1)
    return out * radius, t


def rotation_matrix(rng: np.random.Generator) -> np.ndarray:
    """Uniformly random rotation (QR of a Gaussian matrix with sign fix, det +1)."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def axis_rotation(axis: str, degrees: float) -> np.ndarray:
    a = np.deg2rad(degrees)
    c, s = np.cos(a), np.sin(a)
    if axis == "x":
        return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])
    if axis == "y":
        return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def perturbed_ellipsoid(nu: int, semi_axes, rng: np.random.Generator, n_modes: int = 16,
                        alpha: float = 0.08, clamp: float = 0.15):
    """Seeded protein-like blob: an ellipsoid with a smooth random radial perturbation.

    The unit octasphere is stretched to semi-axes (a, b, c) and every vertex is scaled radially
    by 1 + clip(alpha * f(r_hat), -clamp, clamp), where f is a normalised sum of n_modes plane
    waves sin(k_m . r_hat + phase_m) with |k_m| ~ U[2, 6] and uniformly random directions.
    Centred at the origin; the caller rotates and places it.
    """
    v, t = octasphere(nu, 1.0)
    dirs = rng.standard_normal((n_modes, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    kmag = rng.uniform(2.0, 6.0, n_modes)
    phase = rng.uniform(0.0, 2 * np.pi, n_modes)
    f = np.sin(v @ (dirs * kmag[:, None]).T + phase).sum(1) / np.sqrt(n_modes)
    scale = 1.0 + np.clip(alpha * f, -clamp, clamp)
    v = v * np.asarray(semi_axes, dtype=np.float64)[None, :] * scale[:, None]
    return v, t


def place_at_gap(verts: np.ndarray, direction, sphere_radius: float, gap: float,
                 sphere_center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Translate a blob along a unit direction so its closest vertex is `gap` nm from the sphere.

    Solves min_v |v + t d - c0| - R = gap for the translation t by bisection (the left side
    grows with t once the blob is outside the sphere).
    """
    d = np.asarray(direction, dtype=np.float64)
    d = d / np.linalg.norm(d)
    c0 = np.asarray(sphere_center, dtype=np.float64)

    def dist(t):
        return np.min(np.linalg.norm(verts + t * d - c0, axis=1)) - sphere_radius - gap

    ext = np.max(np.linalg.norm(verts, axis=1))
    lo, hi = sphere_radius, sphere_radius + gap + 2 * ext + 1.0
    if dist(lo) > 0:
        lo = 0.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if dist(mid) > 0:
            hi = mid
        else:
            lo = mid
    return verts + hi * d + c0


def merge_surfaces(surfaces):
    """Concatenate (verts, tris) surfaces; returns verts, tris, per-panel surface id."""
    vs, ts, sid = [], [], []
    off = 0
    for k, (v, t) in enumerate(surfaces):
        vs.append(v)
        ts.append(t + off)
        sid.append(np.full(len(t), k, dtype=np.int32))
        off += len(v)
    return np.concatenate(vs), np.concatenate(ts).astype(np.int32), np.concatenate(sid)
