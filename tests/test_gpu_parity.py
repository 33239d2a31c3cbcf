"""GPU parity: the HIP library (through its C ABI) against the oracle, element by element.

Tolerances: FP64 paths 1e-6 relative on C_ext (the stated bar; observed differences are at the
GMRES tolerance), FP32 paths 1e-4 relative on C_ext.  Matrix-vector products are compared
against the oracle's dense matrix; the bound for each case is stated where it is used.
"""
import numpy as np
import pytest

import oracle
from lspr_inputs import (octasphere, graded_octasphere, perturbed_ellipsoid, place_at_gap,
                         merge_surfaces, eps_silver_drude, workload, EPS_WATER)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_1812_10722_amd import lspr
    assert torch.cuda.is_available()
    return lspr


def _dense_system(surfaces, eps_m, eps_s, k_far=4, k_fine=19, n_k=9, threshold=0.5):
    v, t, sid = merge_surfaces(surfaces)
    V, K = oracle.dense_operators(v, t, k_far, k_fine, n_k, threshold)
    g = oracle.panel_geometry(v, t)
    return v, t, sid, V, K, g


def _rand_x(rng, ncol, n):
    return rng.standard_normal((ncol, 2 * n)) + 1j * rng.standard_normal((ncol, 2 * n))


def sensor_and_blob(nu_s=6, nu_b=5, seed=1):
    rng = np.random.default_rng(seed)
    s = octasphere(nu_s, 8.0)
    bv, bt = perturbed_ellipsoid(nu_b, (1.5, 4.0, 1.5), rng)
    return [s, (place_at_gap(bv, [0.3, 0.2, 1.0], 8.0, 0.6), bt)]


# ----------------------------------------------------------------------------- operator parity
@pytest.mark.parametrize("precision,tol,k_fine", [("fp64", 1e-12, 19), ("fp32", 2e-6, 19),
                                                  ("fp64", 1e-12, 37)])
def test_apply_dense_matches_oracle_matrix(lib, precision, tol, k_fine):
    """y = A x with every far pair summed directly equals the oracle's dense matrix product
    (FP64: rounding only; FP32: single-precision sums with compensated accumulation), with the
    relaxed (19-point) and the strict (37-point, Table quadparams1) near-singular rule."""
    surfs = sensor_and_blob()
    v, t, sid, V, K, g = _dense_system(surfs, None, None, k_fine=k_fine)
    rng = np.random.default_rng(7)
    ncol = 3
    eps_m = np.array([1.7733, 1.80 + 0.01j, 1.0])
    eps_s = np.array([[-3.38 + 0.2j, 2.5], [-2.0 + 0.5j, 2.7 + 0.3j], [4.0, 1.5]])
    x = _rand_x(rng, ncol, len(t))
    geo = lib.Geometry(surfs, method="dense", precision=precision, k_far=4, k_fine=k_fine)
    y = geo.apply(torch.as_tensor(x).cuda(), eps_m, eps_s).cpu().numpy()
    for c in range(ncol):
        A, _ = oracle.assemble_system(V, K, sid, g["normal"], eps_m[c], eps_s[c], [0, 0, 1.0])
        ref = A @ x[c]
        err = np.abs(y[c] - ref).max() / np.abs(ref).max()
        assert err < tol, (precision, c, err)


def test_apply_dense_with_many_near_panels_matches_oracle_matrix(lib):
    """At a small near-singular threshold some targets are near to more than 64 panels, so the
    library builds its near-singular table with a counting and a filling tree walk instead of
    one walk (the case is checked on the oracle's own mask); the dense FP64 product still equals
    the oracle's matrix to rounding."""
    surfs = sensor_and_blob()
    thr = 0.2
    v, t, sid, V, K, g = _dense_system(surfs, None, None, threshold=thr)
    n = len(t)
    mask = oracle.near_singular_mask(g["centroid"], np.arange(n), g["centroid"], g["L"], thr)
    assert mask.sum(axis=1).max() > 64, mask.sum(axis=1).max()
    rng = np.random.default_rng(11)
    eps_m = np.array([1.7733, 1.0])
    eps_s = np.array([[-3.38 + 0.2j, 2.5], [4.0, 1.5]])
    x = _rand_x(rng, 2, n)
    geo = lib.Geometry(surfs, method="dense", precision="fp64", k_far=4, k_fine=19,
                       threshold=thr)
    assert geo.info()["n_near"] == int(mask.sum())
    y = geo.apply(torch.as_tensor(x).cuda(), eps_m, eps_s).cpu().numpy()
    for c in range(2):
        A, _ = oracle.assemble_system(V, K, sid, g["normal"], eps_m[c], eps_s[c], [0, 0, 1.0])
        ref = A @ x[c]
        err = np.abs(y[c] - ref).max() / np.abs(ref).max()
        assert err < 1e-12, (c, err)


def test_geometry_after_a_larger_one_gives_the_same_product(lib):
    """Set-up reuses host tile plans and buffers between geometries: a small treecode geometry
    built again after a larger one gives the same FP32 product, bit for bit, as when it was built
    first."""
    small = sensor_and_blob()
    rng = np.random.default_rng(5)
    eps_m = np.array([1.7733, 1.80 + 0.01j])
    eps_s = np.array([[-3.38 + 0.2j, 2.5], [-2.0 + 0.5j, 2.7 + 0.3j]])
    n = sum(len(t) for _, t in small)
    x = torch.as_tensor(_rand_x(rng, 2, n)).cuda()
    kw = dict(method="treecode", precision="fp32", p=8, theta=0.5, k_far=4, k_fine=19)
    y1 = lib.Geometry(small, **kw).apply(x, eps_m, eps_s).cpu().numpy()
    big = [octasphere(16, 10.0)]
    xb = torch.as_tensor(_rand_x(rng, 2, len(big[0][1]))).cuda()
    lib.Geometry(big, **kw).apply(xb, eps_m, eps_s[:, :1]).cpu().numpy()
    y2 = lib.Geometry(small, **kw).apply(x, eps_m, eps_s).cpu().numpy()
    assert np.array_equal(y1, y2), np.abs(y1 - y2).max()


def test_rhs_matches_oracle(lib):
    surfs = sensor_and_blob()
    v, t, sid, V, K, g = _dense_system(surfs, None, None)
    eps_m = np.array([1.7733, 1.9 + 0.1j])
    eps_s = np.array([[-3.38 + 0.2j, 2.5], [-1.0 + 2.0j, 3.0]])
    e = np.array([0.3, -0.5, 1.2])
    geo = lib.Geometry(surfs, method="dense", precision="fp64")
    b = geo.rhs(eps_m, eps_s, e).cpu().numpy()
    for c in range(2):
        _, ref = oracle.assemble_system(V, K, sid, g["normal"], eps_m[c], eps_s[c], e)
        assert np.abs(b[c] - ref).max() / np.abs(ref).max() < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_treecode_error_falls_with_order(lib, precision):
    """Treecode products converge to the dense product as P grows (MAC theta = 0.5); the
    truncation error of a Taylor expansion of order P scales like theta^(P+1)."""
    v, t = graded_octasphere(16, 10.0)
    V, K = oracle.dense_operators(v, t, 4, 19, 9, 0.5)
    g = oracle.panel_geometry(v, t)
    sid = np.zeros(len(t), int)
    A, _ = oracle.assemble_system(V, K, sid, g["normal"], 1.7733, [-3.38 + 0.2j], [0, 0, 1.0])
    rng = np.random.default_rng(3)
    x = _rand_x(rng, 1, len(t))
    ref = A @ x[0]
    errs = []
    for p in (2, 4, 6, 8, 10):
        geo = lib.Geometry([(v, t)], method="treecode", precision=precision, p=p, theta=0.5,
                           ncrit=8, m2p_min_panels=1)
        assert geo.info()["n_m2p"] > 0
        y = geo.apply(torch.as_tensor(x).cuda(), [1.7733], [[-3.38 + 0.2j]]).cpu().numpy()
        errs.append(np.linalg.norm(y[0] - ref) / np.linalg.norm(ref))
    floor = 1e-13 if precision == "fp64" else 3e-6
    for a, b in zip(errs, errs[1:]):
        assert b < a or b < floor, errs
    assert errs[2] < 2e-4 and errs[-1] < max(1e-5, floor), errs  # P = 6 and P = 10


def test_high_orders_continue_the_convergence(lib):
    """Orders 12 and 15 (the paper's grid-convergence setting, Table treeparams1) run from
    expansion tiles cut into slices of Taylor terms: the FP64 product keeps converging to the
    dense product past P = 10, at the rate theta^(P+1) (theta = 0.5)."""
    v, t = graded_octasphere(16, 10.0)
    V, K = oracle.dense_operators(v, t, 4, 19, 9, 0.5)
    g = oracle.panel_geometry(v, t)
    A, _ = oracle.assemble_system(V, K, np.zeros(len(t), int), g["normal"], 1.7733,
                                  [-3.38 + 0.2j], [0, 0, 1.0])
    rng = np.random.default_rng(5)
    x = _rand_x(rng, 3, len(t))
    errs = []
    for p in (8, 10, 12, 15):
        geo = lib.Geometry([(v, t)], method="treecode", precision="fp64", p=p, theta=0.5,
                           ncrit=8, m2p_min_panels=1)
        assert geo.info()["n_m2p"] > 0
        y = geo.apply(torch.as_tensor(x).cuda(), [1.7733] * 3, [[-3.38 + 0.2j]] * 3).cpu().numpy()
        errs.append(max(np.linalg.norm(y[c] - A @ x[c]) / np.linalg.norm(A @ x[c])
                        for c in range(3)))
        # the FP32 tiles of the same orders (sliced too) agree with the FP64 product
        g32 = lib.Geometry([(v, t)], method="treecode", precision="fp32", p=p, theta=0.5,
                           ncrit=8, m2p_min_panels=1)
        y32 = g32.apply(torch.as_tensor(x).cuda(), [1.7733] * 3,
                        [[-3.38 + 0.2j]] * 3).cpu().numpy()
        assert np.abs(y32 - y).max() / np.abs(y).max() < 3e-6, p
    assert errs[0] > errs[1] > errs[2] > errs[3], errs
    assert errs[3] < 1e-7, errs


@pytest.mark.parametrize("method,ncol,precision", [("treecode", 20, "fp32"), ("dense", 9, "fp32"),
                                                   ("treecode", 64, "fp32"),
                                                   ("treecode", 20, "fp64"), ("treecode", 64, "fp64"),
                                                   ("dense", 9, "fp64")])
def test_matrix_core_kernel_matches_vector_kernel_and_oracle(lib, method, ncol, precision):
    """Products run on matrix cores from precomputed tiles (FP32 or FP64); they must equal the
    vector-ALU kernel (same sums, different order: FP32 3e-6, FP64 1e-12 of the largest
    entry) and the oracle's dense product (treecode: to its truncation error at P = 8)."""
    surfs = sensor_and_blob(10, 7)
    v, t, sid, V, K, g = _dense_system(surfs, None, None)
    rng = np.random.default_rng(11)
    eps_m = np.full(ncol, 1.7733) + 0.01j * rng.standard_normal(ncol)
    eps_s = np.stack([-3.0 + 0.3j + rng.standard_normal(ncol), 2.5 + 0.1j * rng.random(ncol)], 1)
    x = _rand_x(rng, ncol, len(t))
    xt = torch.as_tensor(x).cuda()
    kw = dict(method=method, precision=precision, p=8, theta=0.5)
    mc = lib.Geometry(surfs, **kw)
    vc = lib.Geometry(surfs, matrix_cores=False, **kw)
    y_mc = mc.apply(xt, eps_m, eps_s).cpu().numpy()
    y_vc = vc.apply(xt, eps_m, eps_s).cpu().numpy()
    same = 3e-6 if precision == "fp32" else 1e-12
    for c in (0, ncol // 2, ncol - 1):
        A, _ = oracle.assemble_system(V, K, sid, g["normal"], eps_m[c], eps_s[c], [0, 0, 1.0])
        ref = A @ x[c]
        scale = np.abs(ref).max()
        assert np.abs(y_mc[c] - y_vc[c]).max() / scale < same
        assert np.abs(y_mc[c] - ref).max() / scale < (same if method == "dense" else 1e-4)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_streamed_narrow_products_equal_staged(lib, precision):
    """Products of 1 to 16 wavelengths stream each wave's operands from memory (no LDS): the
    same step partition and summation order as the four-wave form that stages each left factor
    in LDS through registers, so the results are equal bit for bit; both match the oracle's
    dense product to the treecode's truncation error."""
    surfs = sensor_and_blob(10, 7)
    v, t, sid, V, K, g = _dense_system(surfs, None, None)
    kw = dict(method="treecode", precision=precision, p=8, theta=0.5)
    streamed = lib.Geometry(surfs, stream_narrow=True, **kw)
    staged = lib.Geometry(surfs, four_wave=True, **kw)
    rng = np.random.default_rng(17)
    for nl in (1, 5, 8, 9, 12, 16):
        eps_m = np.full(nl, 1.7733) + 0.01j * rng.standard_normal(nl)
        eps_s = np.stack([-3.0 + 0.3j + rng.standard_normal(nl), np.full(nl, 2.5 + 0.1j)], 1)
        xt = torch.as_tensor(_rand_x(rng, nl, len(t))).cuda()
        a = streamed.apply(xt, eps_m, eps_s).cpu().numpy()
        b = staged.apply(xt, eps_m, eps_s).cpu().numpy()
        assert np.array_equal(a, b), (nl, np.abs(a - b).max())
        for c in (0, nl - 1):
            A, _ = oracle.assemble_system(V, K, sid, g["normal"], eps_m[c], eps_s[c], [0, 0, 1.0])
            ref = A @ _to_np(xt[c])
            assert np.abs(a[c] - ref).max() / np.abs(ref).max() < 1e-4


def _to_np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_paired_operator_workgroups_equal_split(lib, precision):
    """Products in eight-wave workgroups that stage each left factor once for both operators:
    each wave's arithmetic is that of the one-operator four-wave workgroups, so the results are
    equal bit for bit (1 to 16 wavelengths: the K-steps split over 4 or 2 waves per column
    group; 17 to 64: one or two column halves)."""
    surfs = sensor_and_blob(10, 7)
    kw = dict(method="treecode", precision=precision, p=8, theta=0.5)
    paired = lib.Geometry(surfs, pair_operators=True, pair_narrow=True, **kw)
    split = lib.Geometry(surfs, four_wave=True, **kw)
    rng = np.random.default_rng(23)
    n = paired.n_panels
    for nl in (1, 5, 8, 9, 16, 17, 20, 40, 64):
        eps_m = np.full(nl, 1.7733) + 0.01j * rng.standard_normal(nl)
        eps_s = np.stack([-3.0 + 0.3j + rng.standard_normal(nl), np.full(nl, 2.5 + 0.1j)], 1)
        xt = torch.as_tensor(_rand_x(rng, nl, n)).cuda()
        a = paired.apply(xt, eps_m, eps_s).cpu().numpy()
        b = split.apply(xt, eps_m, eps_s).cpu().numpy()
        assert np.array_equal(a, b), (nl, np.abs(a - b).max())


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_lds_destination_kernels_against_four_wave_kernels(lib, precision):
    """Products in eight-wave workgroups that read each left factor straight into LDS buffers,
    against the four-wave workgroups that stage it through registers (LSPR_FOUR_WAVE).  Above
    32 wavelengths each wave's operands, K-step order and sums are the same (both column halves
    in one workgroup instead of one each; FP64 in half tiles), so the results are equal bit for
    bit, and at 17-32 both take the four-wave kernel; FP32 products of up to 16 wavelengths split
    the K-steps of a column group over twice as many waves, so their FP32 partial sums differ in
    rounding only: within a few FP32 units of the largest entry (FP64 ones take the four-wave
    kernel)."""
    surfs = sensor_and_blob(10, 7)
    kw = dict(method="treecode", precision=precision, p=8, theta=0.5)
    four = lib.Geometry(surfs, four_wave=True, **kw)
    eight = lib.Geometry(surfs, **kw)
    rng = np.random.default_rng(29)
    n = four.n_panels
    for nl in (1, 5, 8, 9, 12, 16, 17, 24, 32, 33, 40, 41, 48, 57, 64):
        eps_m = np.full(nl, 1.7733) + 0.01j * rng.standard_normal(nl)
        eps_s = np.stack([-3.0 + 0.3j + rng.standard_normal(nl), np.full(nl, 2.5 + 0.1j)], 1)
        xt = torch.as_tensor(_rand_x(rng, nl, n)).cuda()
        a = four.apply(xt, eps_m, eps_s).cpu().numpy()
        b = eight.apply(xt, eps_m, eps_s).cpu().numpy()
        if nl > 16 or precision == "fp64":
            assert np.array_equal(a, b), (nl, np.abs(a - b).max())
        else:
            err = np.abs(a - b).max() / np.abs(a).max()
            assert err < 2e-6, (nl, err)


# ----------------------------------------------------------------------------- full solves
def test_sphere_512_dense_fp64_matches_oracle(lib):
    """The 512-panel silver sphere (lambda = 380 nm) solved by the GPU dense FP64 path equals the
    oracle's LU solution to the GMRES tolerance, at the integration settings of the paper's
    grid-convergence study (Table quadparams1: K = 4, K_fine = 37, N_k = 9)."""
    w = workload("sphere_512")
    assert (w.op["k_far"], w.op["k_fine"], w.op["n_k"]) == (4, 37, 9)
    v, t = w.surfaces[0]
    ref = oracle.solve(v, t, np.zeros(len(t), int), w.lambdas, w.eps_medium, w.eps_surface,
                       w.e_field, k_far=4, k_fine=37, n_k=9, threshold=0.5)
    geo = lib.Geometry(w.surfaces, op=lib.op_params(**w.op))
    out = geo.solve(w.lambdas, w.eps_medium, w.eps_surface, w.e_field, tol=1e-10, restart=100,
                    max_iter=1000, precond=1, want_fields=True)
    assert out["converged"] and out["rel_resid"][0] < 1e-10
    rel = abs(out["cext_sensor"][0] / ref["cext_sensor"][0] - 1)
    assert rel < 1e-6, rel
    assert np.abs(out["p_sensor"][0] - ref["p_sensor"][0]).max() / np.abs(ref["p_sensor"][0]).max() < 1e-7
    phi = out["phi"].cpu().numpy()[0]
    dphi = out["dphi"].cpu().numpy()[0]
    assert np.linalg.norm(phi - ref["phi"][0]) / np.linalg.norm(ref["phi"][0]) < 1e-8
    assert np.linalg.norm(dphi - ref["dphi"][0]) / np.linalg.norm(ref["dphi"][0]) < 1e-8
    an = oracle.cext_sphere_analytic(10.0, 380.0, w.eps_surface[0, 0], w.eps_medium[0])
    assert 0.1 < out["cext_sensor"][0] / an - 1 < 0.4  # 512-panel discretisation error


def test_preconditioner_keeps_solution(lib):
    w = workload("sphere_512")
    geo = lib.Geometry(w.surfaces, method="dense", precision="fp64", k_far=4, k_fine=25)
    a = geo.solve(w.lambdas, w.eps_medium, w.eps_surface, tol=1e-11, restart=200, precond=0)
    b = geo.solve(w.lambdas, w.eps_medium, w.eps_surface, tol=1e-11, restart=200, precond=1)
    assert abs(a["cext_sensor"][0] / b["cext_sensor"][0] - 1) < 1e-9
    assert b["iters"][0] <= a["iters"][0]


@pytest.fixture(scope="module")
def sphere_512_ref():
    w = workload("sphere_512")
    v, t = w.surfaces[0]
    return w, oracle.solve(v, t, np.zeros(len(t), int), w.lambdas, w.eps_medium, w.eps_surface,
                           w.e_field, k_far=4, k_fine=25, n_k=9, threshold=0.5)


@pytest.mark.parametrize("restart", [7, 13])
def test_short_restart_cycles(lib, sphere_512_ref, restart):
    """Cycles of 7 and 13 Arnoldi steps end on a column that is finalised by an inner-product
    pass alone; the restarted solves still meet the tolerance on the true residual and equal
    the oracle's LU solution.  (Cycles of 1 to 5 steps stagnate on this system, as plain
    restarted GMRES does.)"""
    w, ref = sphere_512_ref
    geo = lib.Geometry(w.surfaces, method="dense", precision="fp64", k_far=4, k_fine=25, n_k=9)
    out = geo.solve(w.lambdas, w.eps_medium, w.eps_surface, w.e_field, tol=1e-9,
                    restart=restart, max_iter=4000, precond=1)
    assert out["converged"] and out["rel_resid"][0] <= 1e-9, (out["iters"], out["rel_resid"])
    rel = abs(out["cext_sensor"][0] / ref["cext_sensor"][0] - 1)
    assert rel < 1e-7, rel


@pytest.mark.parametrize("method,precision,tol,p", [("dense", "fp64", 1e-6, 8),
                                                    ("dense", "fp32", 1e-4, 8),
                                                    ("treecode", "fp64", 1e-4, 8),
                                                    ("treecode", "fp64", 1e-6, 15),
                                                    ("treecode", "fp32", 1e-4, 8),
                                                    ("dense", "fp32_refine64", 1e-6, 8),
                                                    ("treecode", "fp32_refine64", 1e-4, 8),
                                                    ("treecode", "fp32_lead64", 1e-4, 8)])
def test_spectrum_matches_oracle(lib, method, precision, tol, p):
    """A spectrum across the Drude resonance (8 wavelengths, 2048-panel sphere, E along x):
    every wavelength's C_ext within the path's bar of the oracle's LU value."""
    v, t = octasphere(16, 10.0)
    lam = np.linspace(360.0, 400.0, 8)
    em = np.full(8, EPS_WATER + 0j)
    es = eps_silver_drude(lam)[:, None]
    e = [1.0, 0.0, 0.0]
    ref = oracle.solve(v, t, np.zeros(len(t), int), lam, em, es, e, k_far=4, k_fine=19)
    geo = lib.Geometry([(v, t)], method=method, precision=precision, p=p, theta=0.5)
    fp32_resid = precision in ("fp32", "fp32_lead64")  # the residual uses FP32 products
    out = geo.solve(lam, em, es, e, tol=1e-6 if fp32_resid else 1e-9, restart=80, max_iter=800)
    assert out["converged"]
    rel = np.abs(out["cext_sensor"] / ref["cext_sensor"] - 1)
    assert rel.max() < tol, rel


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("fp32", 1e-4), ("fp32_refine64", 1e-6)])
def test_sensor_with_analyte_matches_oracle(lib, precision, tol):
    """Two surfaces (Eq. matrix_multi): sensor and total cross-sections and dipoles."""
    surfs = sensor_and_blob(8, 6)
    v, t, sid = merge_surfaces(surfs)
    lam = np.array([375.0, 383.0, 390.0])
    em = np.full(3, EPS_WATER + 0j)
    es = np.stack([eps_silver_drude(lam), np.full(3, 2.5 + 0.1j)], 1)
    ref = oracle.solve(v, t, sid, lam, em, es, [0, 0, 1.0], k_far=4, k_fine=19)
    geo = lib.Geometry(surfs, method="dense", precision=precision)
    out = geo.solve(lam, em, es, [0, 0, 1.0], tol=1e-6 if precision == "fp32" else 1e-10,
                    restart=100, max_iter=1000)
    assert out["converged"]
    for key in ("cext_sensor", "cext_total"):
        rel = np.abs(out[key] / ref[key] - 1)
        assert rel.max() < tol, (key, rel)
    assert np.abs(out["p_total"] - ref["p_total"]).max() / np.abs(ref["p_total"]).max() < 10 * tol


# ----------------------------------------------------------------------------- edge cases
def test_tiny_mesh_and_ragged_batches(lib):
    """8 panels (less than one target chunk), 1, 3 and 67 wavelengths (67 crosses the 64-column
    batch): each wavelength equals the oracle, whatever batch it was solved in."""
    v, t = octasphere(1, 5.0)
    lam = np.linspace(350, 420, 67)
    em = np.full(67, EPS_WATER + 0j)
    es = eps_silver_drude(lam)[:, None]
    ref = oracle.solve(v, t, np.zeros(8, int), lam, em, es, [0, 0, 1.0], k_far=4, k_fine=19)
    geo = lib.Geometry([(v, t)], method="dense", precision="fp64")
    for sel in (slice(0, 1), slice(10, 13), slice(0, 67)):
        out = geo.solve(lam[sel], em[sel], es[sel], tol=1e-12, restart=30)
        assert np.abs(out["cext_total"] / ref["cext_total"][sel] - 1).max() < 1e-9


def test_noconv_reports_and_fills(lib):
    w = workload("sphere_512")
    geo = lib.Geometry(w.surfaces, method="dense", precision="fp64")
    out = geo.solve(w.lambdas, w.eps_medium, w.eps_surface, tol=1e-14, restart=5, max_iter=5,
                    precond=0, allow_noconv=True)
    assert not out["converged"] and out["iters"][0] == 5
    assert 0 < out["rel_resid"][0] < 1 and np.isfinite(out["cext_sensor"][0])


def test_bad_inputs_are_rejected(lib):
    v, t = octasphere(4, 1.0)
    bad = t.copy()
    bad[3, 1] = 10_000
    dv = torch.as_tensor(v).cuda()
    with pytest.raises(lib.LsprError) as e:
        lib.Geometry([(dv, torch.as_tensor(bad).cuda())], method="dense", precision="fp64")
    assert e.value.code == lib.LSPR_E_MESH
    with pytest.raises(lib.LsprError) as e:
        lib.Geometry([(v, t)], method="treecode", p=5)
    assert e.value.code == lib.LSPR_E_INVALID
    geo = lib.Geometry([(v, t)], method="dense", precision="fp64")
    with pytest.raises(lib.LsprError):
        geo.solve([380.0], [1.7733], [[0.0]])  # eps_surface = 0
    # FP32 products cannot certify a residual below 1e-6: such a request is refused up front
    for prec in ("fp32", "fp32_lead64"):
        g32 = lib.Geometry([(v, t)], method="dense", precision=prec)
        with pytest.raises(lib.LsprError) as e:
            g32.solve([380.0], [1.7733], [[-3.38 + 0.2j]], tol=1e-7)
        assert e.value.code == lib.LSPR_E_INVALID
        assert g32.solve([380.0], [1.7733], [[-3.38 + 0.2j]], tol=1e-6)["converged"]


def test_refinement_reaches_fp64_solution(lib):
    """FP32 inner solves with FP64 residuals converge to the FP64 treecode solution: the final
    residual is an FP64 one, and C_ext equals the FP64 solve's to the tolerance."""
    surfs = sensor_and_blob(12, 8)
    lam = np.array([350.0, 384.0, 420.0])
    em = np.full(3, EPS_WATER + 0j)
    es = np.stack([eps_silver_drude(lam), np.full(3, 2.5 + 0j)], 1)
    kw = dict(method="treecode", p=8, theta=0.5)
    ref = lib.Geometry(surfs, precision="fp64", **kw).solve(lam, em, es, tol=1e-10, restart=100,
                                                            max_iter=2000)
    geo = lib.Geometry(surfs, precision="fp32_refine64", **kw)
    for inner in (1e-2, 1e-4):
        out = geo.solve(lam, em, es, tol=1e-9, restart=60, max_iter=3000, inner_tol=inner)
        assert out["converged"] and (out["rel_resid"] <= 1e-9).all(), out["rel_resid"]
        rel = np.abs(out["cext_total"] / ref["cext_total"] - 1)
        assert rel.max() < 1e-7, (inner, rel)


def test_leading_fp64_products(lib):
    """FP64 products for each wavelength's leading Krylov vectors, FP32 after.  With a switch
    level below every residual all products are FP64 and the solve needs no more iterations
    than the FP64 mode; at the default level no more than with FP32 products throughout; both
    give the FP64 solve's C_ext within the tolerance's reach."""
    v, t = octasphere(16, 10.0)
    lam = np.array([370.0, 384.0, 400.0])
    em = np.full(3, EPS_WATER + 0j)
    es = eps_silver_drude(lam)[:, None]
    kw = dict(method="treecode", p=8, theta=0.5)
    gm = dict(tol=1e-6, restart=60, max_iter=600)
    o64 = lib.Geometry([(v, t)], precision="fp64", **kw).solve(lam, em, es, **gm)
    o32 = lib.Geometry([(v, t)], precision="fp32", **kw).solve(lam, em, es, **gm)
    geo = lib.Geometry([(v, t)], precision="fp32_lead64", **kw)
    lead = geo.solve(lam, em, es, **gm)
    all64 = geo.solve(lam, em, es, inner_tol=1e-15, **gm)
    for out in (o64, o32, lead, all64):
        assert out["converged"] and (out["rel_resid"] <= 1e-6).all(), out["rel_resid"]
    assert (lead["iters"] <= o32["iters"] + 1).all(), (lead["iters"], o32["iters"])
    assert (all64["iters"] <= o64["iters"] + 1).all(), (all64["iters"], o64["iters"])
    for out in (lead, all64):
        rel = np.abs(out["cext_total"] / o64["cext_total"] - 1)
        assert rel.max() < 2e-5, rel


def test_autotune_meets_the_bound_and_picks_the_fastest(lib):
    """The autotuner's choice meets its error bound, checked again here with another vector
    against the oracle's dense matrix, and is the fastest timed candidate."""
    v, t = octasphere(12, 10.0)  # 1152 panels
    em = EPS_WATER + 0j
    es = eps_silver_drude(np.array([380.0]))
    bound = 1e-5
    op, entries, ok = lib.lspr_autotune([(v, t)], 8, em, es, max_rel_err=bound)
    assert ok and entries
    timed = [e for e in entries if e["ms_per_product"] >= 0]
    assert timed and all(e["rel_err"] <= bound for e in timed)
    assert all(e["rel_err"] > bound for e in entries if e["ms_per_product"] < 0)
    fastest = min(timed, key=lambda e: e["ms_per_product"])
    assert (op.p, op.ncrit) == (fastest["p"], fastest["ncrit"])
    assert (op.m2p_min_panels, op.flags) == (fastest["m2p_min_panels"], fastest["flags"])
    assert abs(op.theta - fastest["theta"]) < 1e-12 and op.method == lib.LSPR_TREECODE
    # each (theta, N_crit) stops at its first order that meets the bound, orders ascending
    # (the schedule candidates of the second stage repeat the chosen order)
    for th in {e["theta"] for e in entries}:
        for nc in {e["ncrit"] for e in entries}:
            ps = [e["p"] for e in entries if e["theta"] == th and e["ncrit"] == nc]
            assert ps == sorted(ps)
    # the second stage tried the cost threshold both ways and the staged narrow kernel
    sched = [e for e in entries if e["m2p_min_panels"] != 0 or e["flags"] != 0]
    assert {(op.p + 1) ** 2 // 2, 2 * (op.p + 1) ** 2} <= {e["m2p_min_panels"] for e in sched}
    assert any(e["flags"] & lib.LSPR_STREAM_NARROW for e in sched)
    op.precision = lib.LSPR_FP64
    surfs = [(v, t)]
    _, _, sid, V, K, g = _dense_system(surfs, None, None)
    A, _ = oracle.assemble_system(V, K, sid, g["normal"], em, es, [0, 0, 1.0])
    x = _rand_x(np.random.default_rng(5), 1, len(t))
    geo = lib.Geometry(surfs, op=op)
    y = geo.apply(torch.as_tensor(x).cuda(), np.array([em]), es[:, None]).cpu().numpy()
    geo.close()
    ref = A @ x[0]
    assert np.linalg.norm(y[0] - ref) / np.linalg.norm(ref) < 3 * bound


def test_autotuned_schedule_is_no_slower_than_the_fixed_rule(lib):
    """On an 8192-panel sphere at 32 wavelengths, the tuned parameters and kernel schedule
    (bound 1e-6 on the FP64 product, the level the 1e-4 C_ext bar needs near resonance) give an
    FP32 product no slower than the fixed rule the workloads use (P = 8, theta = 0.5, default
    schedule), and the tuned FP64 product meets the bound against the oracle's own rows."""
    v, t = octasphere(32, 10.0)
    em = EPS_WATER + 0j
    es = eps_silver_drude(np.array([384.0]))
    bound, ncol = 1e-6, 32
    op, entries, ok = lib.lspr_autotune([(v, t)], ncol, em, es, max_rel_err=bound, p=8,
                                        theta=0.5, precision="fp32")
    assert ok
    fixed = lib.op_params(p=8, theta=0.5, precision="fp32")
    x = torch.as_tensor(_rand_x(np.random.default_rng(9), ncol, len(t))).cuda()
    ems, ess = np.full(ncol, em), np.repeat(es[:, None], ncol, 0)

    def timed(o):
        geo = lib.Geometry([(v, t)], op=o)
        geo.apply(x, ems, ess)
        best = 1e9
        for _ in range(5):
            lib.lspr_profile_reset()
            lib.lspr_profile_enable(1)
            geo.apply(x, ems, ess)
            torch.cuda.synchronize()
            lib.lspr_profile_enable(0)
            best = min(best, lib.lspr_profile_query("matvec")["total_ms"])
        geo.close()
        return best

    t_fixed, t_tuned = timed(fixed), timed(op)
    assert t_tuned <= 1.1 * t_fixed, (t_tuned, t_fixed, op.p, op.theta, op.ncrit,
                                      op.m2p_min_panels, op.flags)
    # the tuned expansion against the oracle's rows (FP64 product, all columns share eps)
    rng = np.random.default_rng(3)
    rows = np.sort(rng.choice(len(t), 64, replace=False))
    V, K = oracle.operator_rows(v, t, rows, 4, 19, 9, 0.5)
    inner, outer = oracle.system_rows(V, K, rows, np.zeros(len(t), int), em, es)
    o64 = lib.op_params(p=op.p, theta=op.theta, ncrit=op.ncrit, precision="fp64",
                        m2p_min_panels=op.m2p_min_panels)
    geo = lib.Geometry([(v, t)], op=o64)
    y = geo.apply(x[:1], ems[:1], ess[:1]).cpu().numpy()[0]
    geo.close()
    xr = _to_np(x[0])
    ref = np.concatenate([inner @ xr, outer @ xr])
    got = np.concatenate([y[rows], y[len(t) + rows]])
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 3 * bound


@pytest.mark.parametrize("method,precision,tol", [("dense", "fp64", 1e-6),
                                                  ("treecode", "fp32_lead64", 1e-4)])
def test_point_charges_in_an_analyte_match_oracle(lib, method, precision, tol):
    """Three seeded charges inside the analyte (Eq. integral_eq_lspr_system, last row): the
    right-hand side, C_ext and the dipoles equal the oracle's; removing the charges restores
    the charge-free solution."""
    surfs = sensor_and_blob(8, 6)
    v, t, sid = merge_surfaces(surfs)
    blob = surfs[1][0]
    rng = np.random.default_rng(9)
    pos = blob.mean(0)[None, :] + 0.3 * rng.standard_normal((3, 3))
    q = np.array([18.0951, -2 * 18.0951, 0.5 * 18.0951])  # +1, -2, +0.5 e
    charges = (pos, q, np.array([1, 1, 1]))
    lam = np.array([378.0, 386.0])
    em = np.full(2, EPS_WATER + 0j)
    es = np.stack([eps_silver_drude(lam), np.full(2, 2.5 + 0.1j)], 1)
    ref = oracle.solve(v, t, sid, lam, em, es, [0, 0, 1.0], k_far=4, k_fine=19, charges=charges)
    geo = lib.Geometry(surfs, method=method, precision=precision, p=8, theta=0.5)
    geo.set_charges(*charges)
    if method == "dense":  # the right-hand side itself
        g = oracle.panel_geometry(v, t)
        V, K = oracle.dense_operators(v, t, 4, 19, 9, 0.5)
        _, b_ref = oracle.assemble_system(V, K, sid, g["normal"], em[0], es[0], [0, 0, 1.0],
                                          g["centroid"], charges)
        b = geo.rhs(em[:1], es[:1]).cpu().numpy()[0]
        assert np.abs(b - b_ref).max() < 1e-10 * np.abs(b_ref).max()
    fp32 = precision != "fp64"
    kw = dict(tol=1e-6 if fp32 else 1e-10, restart=100, max_iter=1000)
    out = geo.solve(lam, em, es, [0, 0, 1.0], **kw)
    assert out["converged"]
    for key in ("cext_sensor", "cext_total"):
        assert np.abs(out[key] / ref[key] - 1).max() < tol, key
    assert np.abs(out["p_total"] - ref["p_total"]).max() < 10 * tol * np.abs(ref["p_total"]).max()
    geo.set_charges(np.zeros((0, 3)), [], [])
    plain = geo.solve(lam, em, es, [0, 0, 1.0], **kw)
    ref0 = oracle.solve(v, t, sid, lam, em, es, [0, 0, 1.0], k_far=4, k_fine=19)
    assert np.abs(plain["cext_total"] / ref0["cext_total"] - 1).max() < tol
    geo.close()
