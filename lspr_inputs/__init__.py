"""Seeded synthetic inputs (meshes, permittivities, wavelength grids, workload recipes).

This package is shared by the oracle tests and by the GPU path's callers.  It holds no
boundary-element arithmetic: it only produces the arrays both sides receive.
"""
from .meshes import (octasphere, graded_octasphere, perturbed_ellipsoid, place_at_gap,
                     merge_surfaces, rotation_matrix, axis_rotation, octahedral_grid)
from .permittivity import eps_silver_drude, eps_water, wavelength_grid, EPS_WATER
from .workloads import (Workload, workload, WORKLOADS, serving_stream, serving_stream_params,
                        serving_request)

__all__ = [
    "octasphere", "graded_octasphere", "perturbed_ellipsoid", "place_at_gap", "merge_surfaces",
    "rotation_matrix", "axis_rotation", "octahedral_grid", "eps_silver_drude", "eps_water",
    "wavelength_grid", "EPS_WATER", "Workload", "workload", "WORKLOADS", "serving_stream",
    "serving_stream_params", "serving_request",
]
