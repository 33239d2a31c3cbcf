"""Sensing workflow on the GPU path: spectra around the plasmon resonance, the resonance peak
and its shift when analytes are present (the quantities of the paper's sensing experiments),
against the oracle on a small mesh and as a physical trend on a larger one.
"""
import numpy as np
import pytest

import oracle
from lspr_inputs import (octasphere, perturbed_ellipsoid, place_at_gap, merge_surfaces,
                         eps_silver_drude, wavelength_grid, EPS_WATER)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_1812_10722_amd import lspr
    assert torch.cuda.is_available()
    return lspr


def _sensor(nu_s, nu_b, gap, radius=8.0, seed=2):
    rng = np.random.default_rng(seed)
    bv, bt = perturbed_ellipsoid(nu_b, (1.5, 4.0, 1.5), rng)
    return [octasphere(nu_s, radius), (place_at_gap(bv, [0, 0, 1.0], radius, gap), bt),
            (place_at_gap(bv @ np.diag([1.0, -1.0, -1.0]), [0, 0, -1.0], radius, gap), bt)]


def _spectrum(surfs, lam, eps_analyte=2.5):
    em = np.full(len(lam), EPS_WATER + 0j)
    es = np.concatenate([eps_silver_drude(lam)[:, None],
                         np.full((len(lam), len(surfs) - 1), eps_analyte + 0j)], 1)
    return em, es


def test_peak_and_shift_match_oracle(lib):
    """Sensor alone and with two analytes at 1 nm: peak wavelengths and the shift between them
    equal the oracle's (same mesh, same parabola through the spectrum's maximum)."""
    lam = wavelength_grid(372.0, 392.0, 11)
    surfs = _sensor(8, 5, 1.0)
    peaks = {}
    for label, ss in (("alone", surfs[:1]), ("with", surfs)):
        em, es = _spectrum(ss, lam)
        v, t, sid = merge_surfaces(ss)
        ref = oracle.solve(v, t, sid, lam, em, es, [0, 0, 1.0], k_far=4, k_fine=19)
        geo = lib.Geometry(ss, method="dense", precision="fp64")
        out = geo.solve(lam, em, es, [0, 0, 1.0], tol=1e-10, restart=100, max_iter=2000)
        geo.close()
        pg = lib.lspr_resonance_peak(lam, out["cext_sensor"])[0]
        po = lib.lspr_resonance_peak(lam, ref["cext_sensor"])[0]
        assert abs(pg - po) < 1e-4, (label, pg, po)
        peaks[label] = pg
    assert peaks["with"] > peaks["alone"]  # analytes of higher index red-shift the peak


def test_shift_decreases_with_analyte_distance(lib):
    """Treecode FP32 path, sphere of 8192 panels and two analytes of 800 panels at 0.5, 1, 2 nm:
    the red shift of the resonance is positive and falls with distance."""
    lam = wavelength_grid(374.0, 394.0, 21)
    shifts = []
    base = None
    for gap in (None, 0.5, 1.0, 2.0):
        ss = _sensor(32, 10, gap if gap else 1.0)[: 1 if gap is None else 3]
        em, es = _spectrum(ss, lam)
        geo = lib.Geometry(ss, method="treecode", precision="fp32", p=8, theta=0.5)
        out = geo.solve(lam, em, es, [0, 0, 1.0], tol=1e-6, restart=60, max_iter=800)
        geo.close()
        assert out["converged"]
        pk = lib.lspr_resonance_peak(lam, out["cext_sensor"])[0]
        if gap is None:
            base = pk
        else:
            shifts.append(pk - base)
    assert shifts[0] > shifts[1] > shifts[2] > 0.0, shifts
