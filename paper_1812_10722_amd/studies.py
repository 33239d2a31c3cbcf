"""Study drivers on top of the binding, for the paper's convergence and sensing studies
(section "Results": grid convergence of the extinction cross-section, and the resonance shift
caused by analytes for several placements and field directions).  Every number comes from the
HIP library through the C ABI; this module only sequences the calls.
"""
from __future__ import annotations

import math

import numpy as np

from . import lspr as L


def spectrum(surfaces, lambdas, eps_medium, eps_surface, e_field=(0.0, 0.0, 1.0), op=None,
             gmres=None, **op_kw) -> dict:
    """One geometry, one batched solve over `lambdas`; eps_surface [n_lambda][n_surf]."""
    geo = L.Geometry(surfaces, op=op, **op_kw)
    try:
        return geo.solve(lambdas, eps_medium, eps_surface, e_field, gmres=gmres)
    finally:
        geo.close()


def resonance_shift(sensor, analytes, lambdas, eps_medium, eps_sensor, eps_analyte,
                    e_field=(0.0, 0.0, 1.0), op=None, gmres=None, **op_kw) -> dict:
    """Peak of the sensor's C_ext without and with the analytes (parabolic refinement around
    the sampled maximum) and the shift between them.  eps_sensor: [n_lambda]; eps_analyte: one
    value for every analyte."""
    lam = np.asarray(lambdas, dtype=np.float64)
    em = np.broadcast_to(np.asarray(eps_medium, dtype=np.complex128), lam.shape)
    es0 = np.asarray(eps_sensor, dtype=np.complex128)[:, None]
    alone = spectrum([sensor], lam, em, es0, e_field, op=op, gmres=gmres, **op_kw)
    esa = np.concatenate([es0, np.full((len(lam), len(analytes)), complex(eps_analyte))], 1)
    both = spectrum([sensor] + list(analytes), lam, em, esa, e_field, op=op, gmres=gmres,
                    **op_kw)
    p0 = L.lspr_resonance_peak(lam, alone["cext_sensor"])[0]
    p1 = L.lspr_resonance_peak(lam, both["cext_sensor"])[0]
    q1 = L.lspr_resonance_peak(lam, both["cext_total"])[0]
    return {"peak_alone": p0, "peak_with": p1, "shift": p1 - p0, "peak_with_total": q1,
            "shift_total": q1 - p0, "converged": bool(alone["converged"] and both["converged"])}


def grid_convergence(meshes, lam, eps_medium, eps_surface, e_field=(0.0, 0.0, 1.0), op=None,
                     gmres=None, **op_kw) -> dict:
    """C_ext of one wavelength on a sequence of refined single-surface meshes (coarse to fine).
    The observed order in N comes from the last three values (differences of successive
    meshes), and the two finest values are extrapolated with it (Richardson)."""
    n = [int(len(t)) for _, t in meshes]
    c = []
    for surf in meshes:
        out = spectrum([surf], [lam], [eps_medium], [[eps_surface]], e_field, op=op,
                       gmres=gmres, **op_kw)
        c.append(float(out["cext_total"][0]))
    res = {"N": n, "cext": c, "order": None, "richardson": None}
    if len(c) >= 3:
        d1, d2 = abs(c[-2] - c[-3]), abs(c[-1] - c[-2])
        if d1 > 0.0 and d2 > 0.0:
            order = math.log(d1 / d2) / math.log(n[-1] / n[-2])
            res["order"] = order
            res["richardson"] = c[-1] + (c[-1] - c[-2]) / ((n[-1] / n[-2]) ** order - 1.0)
    return res
