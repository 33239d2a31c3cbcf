"""Oracle: a plain, slow, dense-direct CPU boundary-element solver in complex FP64.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check of the package entry file and
the CPU-baseline leg of the benchmark may import or call anything in this package.  The GPU
library never reaches it; it shares no code with the GPU library (no kernels, headers, tables,
helpers or pre/post-processing) and neither side imports the other.

What it computes (Clementi, Cooper & Barba, "Computational nanoplasmonics in the quasistatic
limit for biosensing applications"):

* flat-triangle, piecewise-constant, centroid-collocation discretisation of the Laplace
  single-layer V and double-layer K operators (section "Discretization and linear system",
  Eqs. layers_disc and layers_element);
* three integration regions: semi-analytic singular self-term with N_k Gauss nodes per edge,
  a fine K_fine-point rule inside the near-singular threshold, a K-point rule elsewhere
  (section "Integral evaluation");
* the block systems of Eq. matrix_lspr (one surface) and Eq. matrix_multi (sensor plus
  analytes), assembled densely and solved by LU or by a plain restarted GMRES;
* exterior traces by the interface condition of Eq. electrostatic_scatter, the dipole moment
  as a boundary integral (Eq. dipole_def_gauss_i_final with the sign reading documented in
  `dipole.py`) and the extinction cross-section by the optical theorem (Eq. cext_fwa);
* the analytic sphere cross-section of Eq. an_sol, used as a pin.

Every function is written for a reader checking it against the paper, not for speed.
"""
from .quadrature import triangle_rule, gauss_legendre, RULE_DEGREE
from .geometry import panel_geometry, quadrature_nodes
from .operators import (singular_v_semianalytic, singular_v_closed_form, operator_rows,
                        dense_operators, near_singular_mask)
from .system import assemble_system, system_rows, solve_lu, gmres, solve
from .dipole import exterior_traces, dipole_moment, extinction_cross_section
from .analytic import cext_sphere_analytic

__all__ = [
    "triangle_rule", "gauss_legendre", "RULE_DEGREE", "panel_geometry", "quadrature_nodes",
    "singular_v_semianalytic", "singular_v_closed_form", "operator_rows", "dense_operators",
    "near_singular_mask", "assemble_system", "system_rows", "solve_lu", "gmres", "solve",
    "exterior_traces", "dipole_moment", "extinction_cross_section", "cext_sphere_analytic",
]
