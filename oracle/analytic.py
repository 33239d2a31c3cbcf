"""Analytic extinction cross-section of a small sphere in a lossy host (test infrastructure).

Eq. an_sol (Mishchenko's result, section "Grid convergence and verification with an isolated
silver nanoparticle"):

    C_ext = (4 pi a^3 / k') Im( k^2 (eps_p/eps_m - 1) / (eps_p/eps_m + 2) ),

k = 2 pi sqrt(eps_m) / lambda (principal root), k' = Re k.
"""
from __future__ import annotations

import numpy as np


def cext_sphere_analytic(radius, lam_nm, eps_p, eps_m):
    lam = np.asarray(lam_nm, dtype=np.float64)
    em = np.asarray(eps_m, dtype=np.complex128)
    ratio = np.asarray(eps_p, dtype=np.complex128) / em
    k = 2.0 * np.pi * np.sqrt(em) / lam
    return 4.0 * np.pi * radius ** 3 / k.real * np.imag(k * k * (ratio - 1.0) / (ratio + 2.0))
