"""Host-side checks of the C ABI library (no GPU needed): it loads, exports every function
declared in include/lspr.h, and its host-only entry points behave."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from lspr_inputs import octasphere

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lspr.h")
LIB = os.path.join(ROOT, "paper_1812_10722_amd", "liblspr.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="liblspr.so not built")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(lspr_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = declared_functions()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n


def test_binding_wraps_every_declared_symbol():
    from paper_1812_10722_amd import lspr
    for n in declared_functions():
        assert hasattr(lspr._lib, n)


@pytest.mark.parametrize("n,deg", [(1, 1), (3, 2), (4, 3), (7, 5), (19, 9), (25, 10), (37, 13)])
def test_library_triangle_rules_are_exact(n, deg):
    """The library's own tables (independent of the oracle's) integrate monomials exactly to
    their degree, and no further (closed form a! b! / (a + b + 2)! on the unit triangle)."""
    from paper_1812_10722_amd.lspr import lspr_triangle_rule
    bary, w = lspr_triangle_rule(n)
    assert abs(w.sum() - 1) < 1e-14 and np.allclose(bary.sum(1), 1)
    x, y = bary[:, 1], bary[:, 2]
    for d in range(deg + 1):
        for a in range(d + 1):
            b = d - a
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            assert abs(0.5 * np.sum(w * x ** a * y ** b) / exact - 1) < 1e-13
    d = deg + 1
    miss = max(abs(0.5 * np.sum(w * x ** a * y ** (d - a)) * math.factorial(d + 2)
                   / (math.factorial(a) * math.factorial(d - a)) - 1) for a in range(d + 1))
    assert miss > 1e-8  # the stated degree is the true one


def test_library_gauss_legendre():
    from paper_1812_10722_amd.lspr import lspr_gauss_legendre
    for n in (1, 2, 9, 20):
        t, w = lspr_gauss_legendre(n)
        for k in range(2 * n):
            exact = 0.0 if k % 2 else 2.0 / (k + 1)
            assert abs(np.sum(w * t ** k) - exact) < 1e-13


def test_mesh_validation():
    from paper_1812_10722_amd import lspr
    v, t = octasphere(4, 1.0)
    assert lspr.lspr_mesh_validate([(v, t)]) == lspr.LSPR_OK
    assert lspr.lspr_mesh_validate([(v, t[:, ::-1].copy())]) == lspr.LSPR_E_MESH  # inverted
    assert lspr.lspr_mesh_validate([(v, t[1:])]) == lspr.LSPR_E_MESH              # open
    bad = t.copy()
    bad[0, 0] = len(v) + 5
    assert lspr.lspr_mesh_validate([(v, bad)]) == lspr.LSPR_E_MESH                # index
    assert "surface 0" in lspr._lib.lspr_last_error().decode()
    deg = v.copy()
    deg[t[0, 1]] = deg[t[0, 0]]
    assert lspr.lspr_mesh_validate([(deg, t)]) == lspr.LSPR_E_MESH               # degenerate
    assert lspr.lspr_mesh_validate([]) == lspr.LSPR_E_INVALID


def test_status_strings():
    from paper_1812_10722_amd import lspr
    for code in range(7):
        assert lspr._lib.lspr_status_string(code)


# ----------------------------------------------------------------------------- resonance peak
@pytest.fixture
def lib():
    from paper_1812_10722_amd import lspr
    return lspr


def test_resonance_peak_is_exact_for_a_parabola(lib):
    x = np.array([370.0, 374.5, 377.0, 381.2, 386.0, 392.0])
    y = 5000.0 - 3.0 * (x - 378.3) ** 2
    pl, pc = lib.lspr_resonance_peak(x, y)
    assert abs(pl - 378.3) < 1e-9 and abs(pc - 5000.0) < 1e-6


def test_resonance_peak_of_the_analytic_sphere():
    """On a 2 nm grid the parabola vertex lands within 0.1 nm of the analytic peak (Eq. an_sol
    evaluated on a 0.001 nm grid); the raw grid maximum can be off by up to 1 nm."""
    from paper_1812_10722_amd import lspr
    import oracle
    from lspr_inputs import eps_silver_drude, EPS_WATER
    fine = np.arange(370.0, 400.0, 0.001)
    ref = fine[np.argmax(oracle.cext_sphere_analytic(10.0, fine, eps_silver_drude(fine),
                                                      EPS_WATER))]
    grid = np.arange(371.0, 399.0, 2.0)
    c = oracle.cext_sphere_analytic(10.0, grid, eps_silver_drude(grid), EPS_WATER)
    pl, _ = lspr.lspr_resonance_peak(grid, c)
    assert abs(pl - ref) < 0.1, (pl, ref)


def test_resonance_peak_edges_and_errors(lib):
    x = np.array([1.0, 2.0, 3.0, 4.0])
    assert lib.lspr_resonance_peak(x, np.array([4.0, 3.0, 2.0, 1.0])) == (1.0, 4.0)
    assert lib.lspr_resonance_peak(x, np.array([1.0, 2.0, 3.0, 5.0])) == (4.0, 5.0)
    with pytest.raises(lib.LsprError):
        lib.lspr_resonance_peak(x[::-1], np.ones(4))
    with pytest.raises(lib.LsprError):
        lib.lspr_resonance_peak(x[:2], np.ones(2))


def test_footprint_counts_the_tile_stores_of_each_precision(lib):
    """Host-only arithmetic: a mode that runs products in both precisions holds both tile
    stores, so its estimate exceeds either single-precision mode's; the refinement mode adds
    its four outer vectors on top."""
    gm = lib.gmres_params(tol=1e-5, restart=60, max_iter=600)
    est = {p: lib.lspr_request_footprint(32768, 1, 64, lib.op_params(p=8, precision=p), gm)
           for p in ("fp32", "fp64", "fp32_refine64", "fp32_lead64")}
    assert est["fp32"] < est["fp64"] < est["fp32_lead64"] < est["fp32_refine64"], est
    bad = lib.op_params(p=8)
    bad.precision = 7
    with pytest.raises(lib.LsprError):
        lib.lspr_request_footprint(32768, 1, 64, bad, gm)
