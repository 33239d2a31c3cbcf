"""Pins that tie the oracle to the paper and to mathematics, not to itself.

Each test names what fixes the expected value: a closed form, an identity, a value printed in
the paper, an invariant, or brute force.  None of them re-types the oracle's own formula.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from lspr_inputs import (octasphere, graded_octasphere, merge_surfaces, rotation_matrix,
                         workload)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


# ----------------------------------------------------------------------------- quadrature
@pytest.mark.parametrize("n", sorted(oracle.RULE_DEGREE))
def test_triangle_rule_integrates_monomials_to_its_degree(n):
    """Closed form: on the unit right triangle, integral of x^a y^b = a! b! / (a + b + 2)!."""
    bary, w = oracle.triangle_rule(n)
    assert abs(w.sum() - 1.0) < 1e-14
    assert np.all(bary >= 0) and np.allclose(bary.sum(1), 1.0, atol=1e-15)
    deg = oracle.RULE_DEGREE[n]
    x, y = bary[:, 1], bary[:, 2]  # vertices (0,0), (1,0), (0,1): area 1/2

    def worst(d):
        e = 0.0
        for a in range(d + 1):
            b = d - a
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            e = max(e, abs(0.5 * np.sum(w * x ** a * y ** b) - exact) / exact)
        return e

    for d in range(deg + 1):
        assert worst(d) < 1e-13, (n, d)
    assert worst(deg + 1) > 1e-8  # the stated degree is the true one


def test_gauss_legendre_nodes_are_exact_for_polynomials():
    t, w = oracle.gauss_legendre(9)
    for k in range(18):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * t ** k) - exact) < 1e-14


# ----------------------------------------------------------------------------- geometry
def test_closed_mesh_invariants_and_sphere_area():
    errs = []
    for nu in (4, 8, 16):
        v, t = octasphere(nu, 10.0)
        g = oracle.panel_geometry(v, t)
        assert np.abs((g["area"][:, None] * g["normal"]).sum(0)).max() < 1e-10  # sum A n = 0
        vol = np.sum(g["area"] * np.einsum("ij,ij->i", g["centroid"], g["normal"])) / 3.0
        assert vol > 0 and abs(vol / (4 / 3 * np.pi * 1e3) - 1) < 0.2      # outward, ~sphere
        assert np.allclose(np.linalg.norm(g["normal"], axis=1), 1.0)
        assert np.allclose(g["L"], np.sqrt(2 * g["area"]))
        errs.append(abs(g["area"].sum() / (4 * np.pi * 100.0) - 1))
    assert errs[0] > errs[1] > errs[2]
    assert errs[1] / errs[2] > 3.5  # inscribed-polyhedron area error falls like h^2


# ----------------------------------------------------------------------------- singular V
def test_singular_closed_form_equilateral_centroid():
    """Potential of a unit-density equilateral triangle (side s) at its centroid:
    (1/4pi) * sqrt(3) s ln(2 + sqrt(3)) -- from the elementary integral of sec over +-60 deg."""
    s = 0.7
    tri = np.array([[0, 0, 0], [s, 0, 0], [s / 2, s * np.sqrt(3) / 2, 0]])
    x = tri.mean(0)
    exact = np.sqrt(3) * s * np.log(2 + np.sqrt(3)) / (4 * np.pi)
    assert abs(oracle.singular_v_closed_form(tri, x) - exact) < 1e-15
    assert abs(oracle.singular_v_semianalytic(tri, x, 60) - exact) < 1e-13


def _brute_force_v(tri, x, n=400):
    """Brute force: midpoint-in-angle, exact-in-radius sum over a fine polar fan about x."""
    total = 0.0
    for e in range(3):
        a, b = tri[e], tri[(e + 1) % 3]
        # parametrise the edge finely; each thin wedge (x, p_k, p_k+1) contributes
        # h_k * |dp| / |p_mid - x| to within O(1/n^2)
        s = np.linspace(0, 1, n + 1)
        p = a[None] + s[:, None] * (b - a)[None]
        mid = 0.5 * (p[1:] + p[:-1])
        dl = np.linalg.norm(p[1:] - p[:-1], axis=1)
        n_tri = np.cross(tri[1] - tri[0], tri[2] - tri[0])
        n_tri /= np.linalg.norm(n_tri)
        h = np.dot(a - x, np.cross(b - a, n_tri) / np.linalg.norm(b - a))
        total += h * np.sum(dl / np.linalg.norm(mid - x, axis=1))
    return total / (4 * np.pi)


def _min_angle_deg(tri):
    ang = []
    for k in range(3):
        u, w = tri[(k + 1) % 3] - tri[k], tri[(k + 2) % 3] - tri[k]
        ang.append(np.degrees(np.arccos(np.dot(u, w) / np.linalg.norm(u) / np.linalg.norm(w))))
    return min(ang)


def test_singular_semianalytic_converges_to_closed_form():
    """Brute force pins the closed form; the N_k-node rule converges to it, and on panels of
    mesh quality (all angles >= 30 degrees) N_k = 9 is already within 1e-4."""
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(60):
        tri = rng.standard_normal((3, 3))
        if np.linalg.norm(np.cross(tri[1] - tri[0], tri[2] - tri[0])) < 0.3:
            continue
        x = tri.mean(0)
        exact = oracle.singular_v_closed_form(tri, x)
        assert abs(_brute_force_v(tri, x, 4000) / exact - 1) < 1e-5
        e = [abs(oracle.singular_v_semianalytic(tri, x, n) / exact - 1) for n in (9, 20, 80)]
        assert e[1] <= e[0] + 1e-15 and e[2] < 1e-9
        if _min_angle_deg(tri) >= 30.0:
            assert e[0] < 1e-4
            checked += 1
    assert checked >= 3


# ----------------------------------------------------------------------------- K, V pins
def solid_angle(tri, x):
    """Van Oosterom & Strackee (1983): signed solid angle of a flat triangle seen from x,
    positive when the right-hand normal of (r1, r2, r3) points away from x."""
    R = tri - x[None]
    r = np.linalg.norm(R, axis=1)
    num = np.dot(R[0], np.cross(R[1], R[2]))
    den = r[0] * r[1] * r[2] + np.dot(R[0], R[1]) * r[2] + np.dot(R[0], R[2]) * r[1] \
        + np.dot(R[1], R[2]) * r[0]
    return 2.0 * np.arctan2(num, den)


def test_double_layer_is_minus_solid_angle_over_4pi():
    """K_ij = -Omega_ij / 4pi; sum over a closed surface seen from a surface point is 2 pi."""
    v, t = graded_octasphere(6, 3.0)
    rows = np.array([0, 17, 101, 250])
    V, K = oracle.operator_rows(v, t, rows, k_far=4, k_fine=25, n_k=9, threshold=0.5)
    _, K_coarse = oracle.operator_rows(v, t, rows, k_far=4, k_fine=25, n_k=9, threshold=1e12)
    g = oracle.panel_geometry(v, t)
    for li, i in enumerate(rows):
        om = np.array([solid_angle(v[t[j]], g["centroid"][i]) if j != i else 0.0
                       for j in range(len(t))])
        assert abs(om.sum() - 2 * np.pi) < 1e-12
        d = np.linalg.norm(g["centroid"] - g["centroid"][i], axis=1)
        far = d > 2 * g["L"]
        near = (~far) & (np.arange(len(t)) != i)
        exact = -om / (4 * np.pi)

        def err(k, sel):
            return np.abs(k[sel] - exact[sel]).max() / np.abs(exact[sel]).max()

        # the fine rule on near pairs beats the far rule applied there (region logic)
        assert err(K[li], far) < 5e-3 and err(K[li], near) < 1e-2
        assert err(K[li], near) < 0.5 * err(K_coarse[li], near)
        assert abs(K[li].sum() + 0.5) < 5e-3


@pytest.mark.parametrize("k_fine,bound", [(19, 5e-3), (37, 2e-4)])
def test_near_singular_length_is_the_source_panels(k_fine, bound):
    """Section "Integral evaluation": a panel is integrated with the fine rule when the
    collocation point lies within 2 L of it, L the representative length of the *integrated*
    (source) triangle.  On a mesh with a sharp jump in panel size (a finely meshed sphere
    0.5 nm from a coarse one) the fine-surface targets see large coarse panels well inside
    2 L_source but outside 2 L_target.  Against the exact Van Oosterom-Strackee solid angle,
    K_ij = -Omega_ij / 4 pi, every such pair meets the bound only if the fine rule was used;
    the far rule misses it by an order of magnitude (so measuring the distance in the
    target's L would fail this test)."""
    coarse = octasphere(4, 5.0)
    fine = octasphere(16, 1.5, center=(0.0, 0.0, 5.0 + 0.5 + 1.5))
    v, t, sid = merge_surfaces([coarse, fine])
    g = oracle.panel_geometry(v, t)
    fi = np.flatnonzero(sid == 1)
    rows = fi[np.argsort(g["centroid"][fi, 2])[:12]]  # fine panels facing the coarse sphere
    _, K = oracle.operator_rows(v, t, rows, k_far=4, k_fine=k_fine, n_k=9, threshold=0.5)
    _, K_far = oracle.operator_rows(v, t, rows, k_far=4, k_fine=k_fine, n_k=9, threshold=1e12)
    ci = np.flatnonzero(sid == 0)
    assert g["L"][ci].min() > 5 * g["L"][fi].max()  # the size jump the test relies on
    worst = worst_far = 0.0
    pairs = 0
    for li, i in enumerate(rows):
        d = np.linalg.norm(g["centroid"][ci] - g["centroid"][i], axis=1)
        sel = ci[(d <= 2 * g["L"][ci]) & (d > 2 * g["L"][i])]
        pairs += len(sel)
        exact = np.array([-solid_angle(v[t[j]], g["centroid"][i]) / (4 * np.pi) for j in sel])
        scale = np.abs(exact).max()
        worst = max(worst, np.abs(K[li, sel] - exact).max() / scale)
        worst_far = max(worst_far, np.abs(K_far[li, sel] - exact).max() / scale)
    assert pairs >= 100
    assert worst < bound, worst
    assert worst_far > 10 * bound, worst_far


@pytest.fixture(scope="module")
def graded_ops():
    out = {}
    for nu in (8, 16):
        v, t = graded_octasphere(nu, 10.0)
        V, K = oracle.dense_operators(v, t, 4, 19, 9, 0.5)
        out[nu] = (oracle.panel_geometry(v, t), V, K)
    return out


def test_sphere_spectra_on_graded_mesh(graded_ops):
    """On a sphere of radius a: V 1 = a, K 1 = -1/2, V Y1 = a/3 Y1, K Y1 = -1/6 Y1 (closed
    forms from the l-th eigenvalues a/(2l+1) and -1/(2(2l+1))).  The mesh is graded so that
    V and its transpose differ; the errors must fall with refinement."""
    a = 10.0
    errs = {}
    for nu, (g, V, K) in graded_ops.items():
        y1 = g["centroid"][:, 2] / np.linalg.norm(g["centroid"], axis=1)
        errs[nu] = np.array([np.abs(V.sum(1) / a - 1).max(), np.abs(K.sum(1) + 0.5).max(),
                             np.abs(V @ y1 - a / 3 * y1).max() / (a / 3),
                             np.abs(K @ y1 + y1 / 6).max() / (1 / 6)])
        assert np.abs(V.sum(0) / a - 1).max() > 0.2  # the transpose fails this pin
    assert np.all(errs[16] < errs[8])
    assert np.all(errs[16] < np.array([5e-3, 1e-3, 1e-2, 2e-2]))


# ----------------------------------------------------------------------------- analytic
def test_analytic_formula_reproduces_paper_value():
    """The paper prints C_ext = 1854.48 nm^2 for its case; Eq. an_sol with the printed
    (4-decimal) permittivities gives 1855.13, and the printed value lies inside the spread
    caused by rounding those permittivities."""
    gold = json.load(open(GOLDEN))["sphere_analytic_cext"]
    em = complex(*gold["eps_medium"])
    ep = complex(*gold["eps_particle"])
    c = oracle.cext_sphere_analytic(gold["radius_nm"], gold["lambda_nm"], ep, em)
    assert abs(c - 1855.13) < 0.01
    h = 0.5 * 10.0 ** -gold["printed_digits"]
    vals = [oracle.cext_sphere_analytic(gold["radius_nm"], gold["lambda_nm"],
                                        ep + dr + 1j * di, em + de)
            for dr in (-h, h) for di in (-h, h) for de in (-h, h)]
    assert min(vals) <= gold["cext_nm2"] <= max(vals)


def test_analytic_sphere_512_target():
    w = workload("sphere_512")
    c = oracle.cext_sphere_analytic(10.0, 380.0, w.eps_surface[0, 0], w.eps_medium[0])
    assert abs(c - 4344.96) < 0.01


# ----------------------------------------------------------------------------- full solve
@pytest.fixture(scope="module")
def sphere_solves():
    out = {}
    for nu in (8, 16):
        v, t = octasphere(nu, 8.0)
        gold = json.load(open(GOLDEN))["sphere_analytic_cext"]
        out[nu] = oracle.solve(v, t, np.zeros(len(t), int), [380.0], [complex(*gold["eps_medium"])],
                               [[complex(*gold["eps_particle"])]], [0, 0, 1.0], k_far=4, k_fine=25)
    return out


def test_full_solve_converges_to_analytic_at_first_order(sphere_solves):
    """Grid convergence against Eq. an_sol (the paper's case: a = 8 nm, lambda = 380 nm).
    Paper: 29.86 % and 7.33 % at N = 512 and 2048, observed order 0.98.  Different meshes
    and fine rule, so the same magnitude and order are expected, not the same digits."""
    gold = json.load(open(GOLDEN))
    an = 1855.13
    e = {nu: abs(r["cext_sensor"][0] - an) / an for nu, r in sphere_solves.items()}
    assert 0.15 < e[8] < 0.40 and 0.04 < e[16] < 0.10
    order = np.log(e[8] / e[16]) / np.log(4.0)
    assert abs(order - gold["sphere_grid_convergence_percent_error"]["observed_order"]) < 0.1
    for r in sphere_solves.values():
        assert r["cext_sensor"][0] > 0 and r["rel_resid"][0] < 1e-12


def test_lu_equals_gmres():
    w = workload("sphere_512")
    v, t = w.surfaces[0]
    kw = dict(k_far=4, k_fine=25, n_k=9, threshold=0.5)
    a = oracle.solve(v, t, np.zeros(len(t), int), w.lambdas, w.eps_medium, w.eps_surface,
                     w.e_field, method="lu", **kw)
    b = oracle.solve(v, t, np.zeros(len(t), int), w.lambdas, w.eps_medium, w.eps_surface,
                     w.e_field, method="gmres", tol=1e-12, restart=50, **kw)
    x_a = np.concatenate([a["phi"][0], a["dphi"][0]])
    x_b = np.concatenate([b["phi"][0], b["dphi"][0]])
    assert np.linalg.norm(x_a - x_b) / np.linalg.norm(x_a) < 1e-9
    assert b["iters"][0] > 10 and b["rel_resid"][0] < 1e-11


# ----------------------------------------------------------------------------- invariants
def _solve_one(v, t, sid, e, eps_s, lam=380.0, em=1.7733):
    return oracle.solve(v, t, sid, [lam], [em], [eps_s], e, k_far=4, k_fine=19)


def test_rotation_field_magnitude_and_permutation_invariance():
    v, t = graded_octasphere(6, 10.0)
    sid = np.zeros(len(t), int)
    eps = [-3.38 + 0.2j]
    base = _solve_one(v, t, sid, [0, 0, 1.0], eps)["cext_sensor"][0]
    R = rotation_matrix(np.random.default_rng(3))
    rot = _solve_one(v @ R.T, t, sid, R @ np.array([0, 0, 1.0]), eps)["cext_sensor"][0]
    big = _solve_one(v, t, sid, [0, 0, -7.5], eps)["cext_sensor"][0]
    perm = np.random.default_rng(4).permutation(len(t))
    prm = _solve_one(v, t[perm], sid, [0, 0, 1.0], eps)["cext_sensor"][0]
    for c in (rot, big, prm):
        assert abs(c / base - 1) < 1e-10


def test_octahedral_symmetry_of_octasphere():
    v, t = octasphere(6, 10.0)
    sid = np.zeros(len(t), int)
    c = [_solve_one(v, t, sid, e, [-3.38 + 0.2j])["cext_sensor"][0]
         for e in ([1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0])]
    assert max(c) / min(c) - 1 < 1e-10


def test_two_sphere_coupling_matches_coupled_dipoles():
    """Pins the cross-surface blocks of Eq. matrix_multi: two identical spheres at distance D
    in a static field.  Point-dipole theory gives the enhancement 1 / (1 - 2 beta a^3/D^3)
    along the axis and 1 / (1 + beta a^3/D^3) across it (beta = (e - 1)/(e + 2)); higher
    multipoles and the 512-panel meshes add about 1 %.  Without coupling the ratio is 1."""
    eps, a, D = 1000.0, 1.0, 3.0
    beta = (eps - 1) / (eps + 2)
    v1, t1 = octasphere(8, a)
    single = _solve_one(v1, t1, np.zeros(len(t1), int), [0, 0, 1.0], [eps], 500.0, 1.0)
    q1 = single["p_total"][0][2].real
    assert abs(q1 / (4 * np.pi * a ** 3 * beta) - 1) < 0.05
    for axis, pred in (("z", 1 / (1 - 2 * beta / D ** 3)), ("x", 1 / (1 + beta / D ** 3))):
        d = np.zeros(3)
        d["xyz".index(axis)] = D / 2
        v, t, sid = merge_surfaces([(v1 - d, t1), (v1 + d, t1)])
        r = _solve_one(v, t, sid, [0, 0, 1.0], [eps, eps], 500.0, 1.0)
        q = r["p_total"][0]
        assert abs(q[2].real / (2 * q1) - pred) < 0.015
        assert abs(q[0]) + abs(q[1]) < 1e-9 * abs(q[2])   # mirror symmetry of the pair
        # each sphere's own dipole is half of the pair's
        assert abs(r["p_sensor"][0][2] / q[2] - 0.5) < 1e-9


def test_index_matched_analyte_is_nearly_invisible():
    """An analyte with eps = eps_m scatters nothing: the sensor's cross-section returns to the
    isolated value up to discretisation error, and much closer than with eps = 2.5."""
    vs, ts = octasphere(6, 8.0)
    vb, tb = octasphere(5, 2.0)
    vb = vb + np.array([0, 0, 11.0])
    v, t, sid = merge_surfaces([(vs, ts), (vb, tb)])
    em = 1.7733
    iso = _solve_one(vs, ts, np.zeros(len(ts), int), [0, 0, 1.0], [-3.38 + 0.2j])["cext_sensor"][0]
    matched = _solve_one(v, t, sid, [0, 0, 1.0], [-3.38 + 0.2j, em])["cext_sensor"][0]
    loaded = _solve_one(v, t, sid, [0, 0, 1.0], [-3.38 + 0.2j, 2.5 + 0j])["cext_sensor"][0]
    assert abs(matched / iso - 1) < 0.2 * abs(loaded / iso - 1)


def test_system_rows_are_rows_of_the_assembled_system():
    """The row-subset form of Eq. matrix_multi used for sampled parity at full size equals the
    dense assembly (itself pinned by the solves above) on a two-surface mesh."""
    rng = np.random.default_rng(4)
    s = octasphere(4, 8.0)
    bv, bt = octasphere(3, 3.0)
    surfs = [s, (bv + np.array([0.0, 0.0, 12.0]), bt)]
    v, t, sid = merge_surfaces(surfs)
    V, K = oracle.dense_operators(v, t, 4, 19, 9, 0.5)
    g = oracle.panel_geometry(v, t)
    eps_m, eps_s = 1.7733 + 0.01j, np.array([-3.4 + 0.2j, 2.5 + 0.1j])
    A, _ = oracle.assemble_system(V, K, sid, g["normal"], eps_m, eps_s, [0, 0, 1.0])
    rows = rng.choice(len(t), 17, replace=False)
    inner, outer = oracle.system_rows(V[rows], K[rows], rows, sid, eps_m, eps_s)
    N = len(t)
    assert np.array_equal(inner, A[rows]) and np.array_equal(outer, A[N + rows])


def test_point_charge_at_the_centre_of_a_dielectric_sphere():
    """Closed form (Born's ion): a charge q at the centre of a sphere of radius R and
    permittivity eps_in in a medium eps_out.  Outside, phi = q / (4 pi eps_out r); inside,
    phi = q / (4 pi eps_in r) + const, so on the surface phi = q / (4 pi eps_out R) and the
    interior normal derivative is -q / (4 pi eps_in R^2).  The charge's response is the
    difference of solves with and without it (the system is linear); the flat-panel error
    falls at second order in the panel size."""
    R, eps_in, eps_out, q = 10.0, 2.0 + 0.0j, 1.7733 + 0.0j, 3.0
    errs = []
    for nu in (6, 12):
        v, t = octasphere(nu, R)
        sid = np.zeros(len(t), int)
        kw = dict(lambdas=[500.0], eps_medium=[eps_out], eps_surface=[[eps_in]],
                  e_field=[0.0, 0.0, 1.0])
        with_q = oracle.solve(v, t, sid, charges=(np.zeros((1, 3)), np.array([q]),
                                                  np.array([0])), **kw)
        without = oracle.solve(v, t, sid, **kw)
        phi = with_q["phi"][0] - without["phi"][0]
        dphi = with_q["dphi"][0] - without["dphi"][0]
        area = oracle.panel_geometry(v, t)["area"]
        phi_avg = np.sum(area * phi) / area.sum()
        dphi_avg = np.sum(area * dphi) / area.sum()
        e_phi = abs(phi_avg / (q / (4 * np.pi * eps_out * R)) - 1)
        e_dphi = abs(dphi_avg / (-q / (4 * np.pi * eps_in * R * R)) - 1)
        errs.append((e_phi, e_dphi))
    assert errs[1][0] < 0.01 and errs[1][1] < 0.01, errs
    assert errs[1][0] < errs[0][0] / 2.5 and errs[1][1] < errs[0][1] / 2.5, errs
