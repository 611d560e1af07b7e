"""Seeded synthetic inputs for the spherical tree code.

This module builds the particle sets, quadrature weights and initial vorticity
fields that both the CPU oracle and the GPU library consume.  It contains no
part of the summation method itself (no kernels, no tree, no interpolation):
only the input recipes of the paper's test cases.

* ``icosahedral_grid``  -- vertices of an iteratively refined icosahedron
  (Sec. 2, the particle set below the discrete BVE system).
* ``node_patch_areas`` / ``uniform_areas`` -- quadrature weights A_j.
* ``rossby_haurwitz``, ``gaussian_vortex`` ... -- initial vorticity fields
  (Sec. 4, Rossby-Haurwitz wave and Gaussian vortex test cases).
* ``random_rotation``, ``random_sphere_points`` -- seeded geometry helpers.
"""

from .grids import (
    icosahedron_vertices,
    icosahedral_grid,
    grid_size,
    uniform_areas,
    node_patch_areas,
    random_rotation,
    random_sphere_points,
    clustered_sphere_points,
    subset_indices,
)
from .fields import (
    OMEGA_EARTH_S,
    OMEGA_EARTH_DAY,
    rossby_haurwitz,
    rossby_haurwitz_paper,
    gaussian_vortex,
    gaussian_vortex_paper,
    gaussian_pair,
    polar_vortex,
    lonlat,
)
from .workloads import make_workload, make_ensemble, make_member, make_gate_training_input, WORKLOADS

__all__ = [
    "icosahedron_vertices", "icosahedral_grid", "grid_size", "uniform_areas",
    "node_patch_areas", "random_rotation", "random_sphere_points",
    "clustered_sphere_points", "subset_indices", "OMEGA_EARTH_S",
    "OMEGA_EARTH_DAY", "rossby_haurwitz", "rossby_haurwitz_paper",
    "gaussian_vortex", "gaussian_vortex_paper", "gaussian_pair", "polar_vortex", "lonlat",
    "make_workload", "make_ensemble", "make_member", "make_gate_training_input", "WORKLOADS",
]
