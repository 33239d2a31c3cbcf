"""The five synthetic workloads (shapes and sizes of the paper's experiments).

Each recipe is deterministic: meshes are seeded with numpy's PCG64 generator and the silver
permittivity is the seed-free Drude formula.  The paper's protein (BSA) meshes and measured
permittivity tables are not available; perturbed ellipsoids of BSA-like size (14 x 4 x 4 nm,
about 30-45 k triangles) and the Drude model stand in for them.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .meshes import (octasphere, perturbed_ellipsoid, place_at_gap, rotation_matrix,
                     axis_rotation)
from .permittivity import eps_silver_drude, wavelength_grid, EPS_WATER


@dataclass
class Workload:
    name: str
    surfaces: list                      # [(verts [n_v,3] f64, tris [n_t,3] i32)], surface 0 = sensor
    lambdas: np.ndarray                 # [n_lambda] nm
    eps_medium: np.ndarray              # [n_lambda] complex
    eps_surface: np.ndarray             # [n_lambda, n_surf] complex
    e_field: np.ndarray = field(default_factory=lambda: np.array([0.0, 0.0, 1.0]))
    op: dict = field(default_factory=dict)      # quadrature / treecode / precision parameters
    gmres: dict = field(default_factory=dict)   # tol, restart, max_iter
    seed: int | None = None
    # treecode parameters and kernel schedule chosen by the library's autotuner before the
    # solve, under this bound on the FP64 product error at this batch width (None: op as given)
    tune: dict | None = None

    @property
    def n_panels(self) -> int:
        return int(sum(len(t) for _, t in self.surfaces))


def _sphere_case(nu, radius, lambdas, eps_p=None):
    lam = np.asarray(lambdas, dtype=np.float64)
    em = np.full(len(lam), EPS_WATER + 0j)
    ep = eps_silver_drude(lam) if eps_p is None else np.full(len(lam), complex(eps_p))
    return [octasphere(nu, radius)], lam, em, ep[:, None]


def sphere_512():
    """Isolated silver sphere R = 10 nm, 512 panels, 380 nm, eps_p = -3.38+0.20i, dense FP64,
    with the integration settings of the paper's grid-convergence study (Table quadparams1:
    K = 4, K_fine = 37, N_k = 9)."""
    surfs, lam, em, es = _sphere_case(8, 10.0, [380.0], eps_p=-3.38 + 0.20j)
    return Workload("sphere_R10_N512_lambda380_dense_fp64", surfs, lam, em, es,
                    op=dict(k_far=4, k_fine=37, n_k=9, threshold=0.5, method="dense",
                            precision="fp64"),
                    gmres=dict(tol=1e-8, restart=100, max_iter=1000))


def sphere_32k_sweep(n_lambda=64, nu=64, p=8, theta=0.5, tol=1e-5):
    """Silver sphere R = 10 nm, 32768 panels, 64 wavelengths 350-420 nm, treecode, FP32 kernels.

    The configured expansion (theta = 0.5, P = 6) misses 1e-4 relative C_ext near resonance
    (measured max 6.2e-4 against FP64 dense); P = 8 at theta = 0.5 is the lowest order that
    meets it (measured max 7e-6), so it is the default here.  GMRES stops at a relative
    residual of 1e-5, which keeps every C_ext within 1e-5 of the FP64 value (measured max
    9.5e-6), a tenfold margin under the 1e-4 target.  Products: FP64 for each wavelength's
    leading Krylov vectors (residual estimate above 0.3), FP32 after; with FP32 products
    throughout the solves need 45 iterations on average instead of 29."""
    surfs, lam, em, es = _sphere_case(nu, 10.0, wavelength_grid(350.0, 420.0, n_lambda))
    return Workload(f"sphere_R10_N{8 * nu * nu}_sweep{n_lambda}_350-420nm_treecode_fp32lead64",
                    surfs, lam, em, es,
                    op=dict(k_far=4, k_fine=19, n_k=9, threshold=0.5, method="treecode",
                            p=p, theta=theta, ncrit=0, precision="fp32_lead64"),
                    gmres=dict(tol=tol, restart=60, max_iter=600))


def sensor_two_analytes(seed=3, nu_sphere=71, nu_blob=61, gap=1.0, n_lambda=32, axis="z"):
    """Sphere R = 8 nm plus two perturbed 14x4x4 nm ellipsoids at +/- axis, 1 nm gap, eps 2.5;
    FP32 products inside FP64-residual refinement, treecode settings from the autotuner."""
    rng = np.random.default_rng(seed)
    sphere = octasphere(nu_sphere, 8.0)
    bv, bt = perturbed_ellipsoid(nu_blob, (2.0, 7.0, 2.0), rng)  # long axis along y
    d = {"x": np.array([1.0, 0, 0]), "y": np.array([0, 1.0, 0]), "z": np.array([0, 0, 1.0])}[axis]
    # the second blob is the first turned 180 degrees about an axis normal to the placement axis
    flip = axis_rotation("y" if axis != "y" else "x", 180.0)
    b1 = place_at_gap(bv, d, 8.0, gap)
    b2 = place_at_gap(bv @ flip.T, -d, 8.0, gap)
    lam = wavelength_grid(375.0, 395.0, n_lambda)
    em = np.full(len(lam), EPS_WATER + 0j)
    es = np.stack([eps_silver_drude(lam), np.full(len(lam), 2.5 + 0j),
                   np.full(len(lam), 2.5 + 0j)], 1)
    return Workload(f"sensor_R8_N{len(sphere[1])}+2x{len(bt)}_gap{gap}_{axis}_sweep{n_lambda}",
                    [sphere, (b1, bt), (b2, bt)], lam, em, es,
                    op=dict(k_far=4, k_fine=19, n_k=9, threshold=0.5, method="treecode",
                            p=8, theta=0.5, ncrit=0, precision="fp32_refine64"),
                    gmres=dict(tol=1e-6, restart=60, max_iter=1200, inner_tol=1e-3), seed=seed,
                    tune=dict(max_rel_err=1e-6, n_cols=n_lambda))


def _place_blobs(rng, n_blobs, nu_blob, radius, gap_range, semi=(2.0, 7.0, 2.0),
                 min_sep=0.5):
    """Seeded blobs around a sphere at gaps drawn from gap_range, each at least min_sep nm from
    every blob already placed (exact vertex distances, k-d tree)."""
    from scipy.spatial import cKDTree
    placed = []  # k-d trees of placed blobs' vertices
    out = []
    for _ in range(n_blobs):
        bv, bt = perturbed_ellipsoid(nu_blob, semi, rng)
        bv = bv @ rotation_matrix(rng).T
        for _attempt in range(1000):
            d = rng.standard_normal(3)
            d /= np.linalg.norm(d)
            g = rng.uniform(*gap_range)
            v = place_at_gap(bv, d, radius, g)
            if all(tree.query(v, k=1)[0].min() > min_sep for tree in placed):
                placed.append(cKDTree(v))
                out.append((v, bt))
                break
        else:
            raise RuntimeError("could not place blob without overlap")
    return out


def large_sensor(seed=4, nu_sphere=128, nu_blob=75, n_blobs=8, n_lambda=16):
    """Sphere R = 10 nm (131072 panels) plus 8 seeded blobs of 45000 panels, gaps 0.5-3 nm."""
    rng = np.random.default_rng(seed)
    surfs = [octasphere(nu_sphere, 10.0)] + _place_blobs(rng, n_blobs, nu_blob, 10.0, (0.5, 3.0))
    lam = wavelength_grid(375.0, 395.0, n_lambda)
    em = np.full(len(lam), EPS_WATER + 0j)
    es = np.concatenate([eps_silver_drude(lam)[:, None],
                         np.full((len(lam), n_blobs), 2.5 + 0j)], 1)
    n = sum(len(t) for _, t in surfs)
    return Workload(f"large_sensor_R10_N{n}_{n_blobs}blobs_sweep{n_lambda}", surfs, lam, em, es,
                    op=dict(k_far=4, k_fine=19, n_k=9, threshold=0.5, method="treecode",
                            p=8, theta=0.5, ncrit=0, precision="fp32_refine64"),
                    gmres=dict(tol=1e-6, restart=60, max_iter=1200, inner_tol=1e-3), seed=seed,
                    tune=dict(max_rel_err=1e-6, n_cols=n_lambda))


def serving_stream_params(seed=5, n_requests=2000, rate_per_s=1.0, nu_range=(16, 128),
                          blob_nu_range=(25, 75), max_blobs=4, max_lambda=64):
    """The draws of the seeded Poisson request stream, without meshes (cheap):
    (arrival_s, k, nu, n_blobs, nu_blob, wavelengths) per request."""
    rng = np.random.default_rng(seed)
    t = 0.0
    for k in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        nu = int(rng.integers(nu_range[0], nu_range[1] + 1))
        nb = int(rng.integers(0, max_blobs + 1))
        nub = int(rng.integers(blob_nu_range[0], blob_nu_range[1] + 1))
        nl = int(rng.integers(1, max_lambda + 1))
        lam = np.sort(rng.uniform(350.0, 420.0, nl))
        yield t, k, nu, nb, nub, lam


def serving_request(seed, k, nu, nb, nub, lam):
    """Request k of the stream from its draws (the blobs come from a generator of its own, so
    requests can be built in any order or in parallel)."""
    nl = len(lam)
    sub = np.random.default_rng([seed, k])
    surfs = [octasphere(nu, 10.0)] + (_place_blobs(sub, nb, nub, 10.0, (0.5, 3.0))
                                      if nb else [])
    em = np.full(nl, EPS_WATER + 0j)
    es = np.concatenate([eps_silver_drude(lam)[:, None], np.full((nl, nb), 2.5 + 0j)], 1)
    return Workload(f"req{k}", surfs, lam, em, es,
                    op=dict(k_far=4, k_fine=19, n_k=9, threshold=0.5, method="treecode",
                            p=8, theta=0.5, ncrit=0, precision="fp32_refine64"),
                    gmres=dict(tol=1e-6, restart=60, max_iter=1200, inner_tol=1e-3),
                    seed=seed)


def serving_stream(seed=5, n_requests=2000, **kw):
    """Seeded Poisson request stream: (arrival_s, Workload) pairs, generated lazily.

    Requests solve with FP32 products and FP64 residuals (iterative refinement): analytes at
    sub-nanometre gaps make the systems ill-conditioned near resonance, where GMRES on FP32
    products alone needs several times more iterations."""
    for t, k, nu, nb, nub, lam in serving_stream_params(seed, n_requests, **kw):
        yield t, serving_request(seed, k, nu, nb, nub, lam)


WORKLOADS = {
    "sphere_512": sphere_512,
    "sphere_32k_sweep": sphere_32k_sweep,
    "sensor_two_analytes": sensor_two_analytes,
    "large_sensor": large_sensor,
}


def workload(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)
