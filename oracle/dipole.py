"""Exterior traces, dipole moment and extinction cross-section (test infrastructure only).

Exterior traces from the interface conditions of Eq. electrostatic_scatter (and their
multi-surface form, Eq. electrostatic_scatter_prot_sen): the potential is continuous and
    eps_s dphi_in/dn - eps_m dphi_out/dn = (eps_m - eps_s) dphi_inc/dn,
so on a panel of surface s
    phi_out = phi,    psi_out = (eps_s / eps_m) psi - ((eps_m - eps_s) / eps_m) g.

Dipole moment (section "Boundary integral expression of the dipole moment").  Reading of the
sign: Green's second identity for phi_out and x_k over the exterior region, closed by a large
sphere on which phi_out tends to p . r_hat / (4 pi eps_m r^2), gives with outward normals

    p_k / eps_m = surface integral of (phi_out n_k - x_k dphi_out/dn) dA,

the opposite sign to the printed Eq. dipole_def_gauss_i_final.  With the printed sign the
exact sphere solution would give a negative cross-section; the analytic sphere (Eq. an_sol)
pins the reading.  With constant values on a flat panel the integral of x over the panel is
Area * centroid exactly.

Extinction (Eqs. scat_efield_long_range, scat_efield_fwa and cext_fwa): in the forward
direction r_hat is normal to the polarisation e, so e . F = k^2 (e . p) / (4 pi eps_m) and

    C_ext = (4 pi / k') Im[e . F / |E|] = Im[k^2 (E . p / eps_m)] / (k' |E|^2),

with k = 2 pi n / lambda, n = sqrt(eps_m) (principal root) and k' = Re k.  Writing E . p
over |E|^2 keeps C_ext independent of the magnitude and sign of the field.
"""
from __future__ import annotations

import numpy as np


def exterior_traces(phi, psi, g, eps_panel, eps_m):
    """(phi_out, psi_out) per panel from interior-side unknowns and g = dphi_inc/dn."""
    return phi, (eps_panel / eps_m) * psi - ((eps_m - eps_panel) / eps_m) * g


def dipole_moment(area, normal, centroid, phi_out, psi_out, mask=None):
    """q = p / eps_m = sum_i A_i (phi_out_i n_i - c_i psi_out_i) over the masked panels."""
    if mask is None:
        mask = np.ones(len(area), dtype=bool)
    a = area[mask]
    return (a[:, None] * (phi_out[mask][:, None] * normal[mask]
                          - centroid[mask] * psi_out[mask][:, None])).sum(0)


def extinction_cross_section(q, e_field, lam_nm, eps_m):
    """C_ext (nm^2) from q = p / eps_m for incident field vector e_field at wavelength lam_nm."""
    e = np.asarray(e_field, dtype=np.float64)
    k = 2.0 * np.pi * np.sqrt(complex(eps_m)) / lam_nm
    return float(np.imag(k * k * np.dot(e, q)) / (k.real * np.dot(e, e)))
