"""Seed-free material models used as synthetic inputs.

The paper interpolates measured tables for silver and water (section "Grid convergence and
verification with an isolated silver nanoparticle"); those tables are not available here, so a
fixed Drude formula stands in for silver and a constant stands in for water.
"""
from __future__ import annotations

import numpy as np

HC_EV_NM = 1239.841984  # photon energy (eV) times wavelength (nm)

# Drude parameters chosen so that eps(380 nm) reproduces the paper's silver value
# -3.3877 + 0.1922i to four decimals.
DRUDE_EPS_INF = 5.0
DRUDE_HBAR_OMEGA_P = 9.4519  # eV
DRUDE_HBAR_GAMMA = 0.07476   # eV

EPS_WATER = 1.7733


def eps_silver_drude(lambda_nm):
    """Complex relative permittivity eps(lambda) = eps_inf - wp^2 / (w^2 + i gamma w)."""
    w = HC_EV_NM / np.asarray(lambda_nm, dtype=np.float64)
    return DRUDE_EPS_INF - DRUDE_HBAR_OMEGA_P ** 2 / (w * w + 1j * DRUDE_HBAR_GAMMA * w)


def eps_water(lambda_nm):
    return np.full(np.shape(lambda_nm), EPS_WATER + 0j)


def wavelength_grid(lo: float, hi: float, n: int):
    """n wavelengths evenly spaced on [lo, hi] (inclusive); a single point gives lo."""
    if n == 1:
        return np.array([float(lo)])
    return lo + (hi - lo) * np.arange(n) / (n - 1)
