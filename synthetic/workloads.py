"""Named workloads: seeded particle set + vorticity + areas + method settings.

Every workload is synthetic (the paper's test cases are all analytic initial
conditions; no dataset exists or is needed):

* ``rh4_l5``   N = 10242 (icosahedron refined 5 times), A = 4 pi / N,
               Rossby-Haurwitz n = 4, omega = K = 7.848e-6 s^-1; theta = 0.7,
               d = 8, FP64.
* ``gv_l8``    N = 655362 (level 8), A = 4 pi / N, Gaussian vortex of width
               0.1 at a seeded centre (seed 2) plus U(-1e-3, 1e-3) noise; the
               precision (FP32) form; error measured on 4096 seeded targets.
* ``rh4_l7``   N = 163842 (level 7), node-patch areas, RH n = 4; RK4 with
               dt = 1800 s.
* ``gvpair_l9`` N = 2621442 (level 9), RH n = 4 background plus a +/- vortex
               pair of amplitude 4 pi per day.
"""

import numpy as np

from .grids import (icosahedral_grid, uniform_areas, node_patch_areas,
                    subset_indices, random_rotation)
from .fields import rossby_haurwitz, gaussian_vortex, gaussian_pair

WORKLOADS = ("rh4_l5", "gv_l8", "rh4_l7", "gvpair_l9")


def make_workload(name, level=None):
    """Return a dict with x (N,3), zeta (N,), area (N,), subset (indices) and
    the workload's method settings.  `level` overrides the grid level (used to
    build the same recipe at a smaller size)."""
    if name == "rh4_l5":
        L = 5 if level is None else level
        x = icosahedral_grid(L)
        n = len(x)
        return dict(name=name, x=x, zeta=rossby_haurwitz(x, 4),
                    area=uniform_areas(n), subset=np.arange(n),
                    theta=0.7, degree=8, seed=0)
    if name == "gv_l8":
        L = 8 if level is None else level
        x = icosahedral_grid(L)
        n = len(x)
        return dict(name=name, x=x, zeta=gaussian_vortex(x, seed=2),
                    area=uniform_areas(n), subset=subset_indices(n, 4096, 2),
                    theta=0.7, degree=8, seed=2)
    if name == "rh4_l7":
        L = 7 if level is None else level
        x, faces = icosahedral_grid(L, return_faces=True)
        return dict(name=name, x=x, zeta=rossby_haurwitz(x, 4),
                    area=node_patch_areas(x, faces),
                    subset=subset_indices(len(x), 4096, 3),
                    theta=0.7, degree=8, seed=3, dt=1800.0, steps=480)
    if name == "gvpair_l9":
        L = 9 if level is None else level
        x = icosahedral_grid(L)
        n = len(x)
        z = rossby_haurwitz(x, 4) + gaussian_pair(x, seed=5)
        return dict(name=name, x=x, zeta=z, area=uniform_areas(n),
                    subset=subset_indices(n, 4096, 5),
                    theta=0.7, degree=10, seed=5)
    if name == "rotated_rh":
        # an icosahedral grid under a random rotation (no particle on a
        # tree edge), used for tie-free parity cases
        L = 4 if level is None else level
        q = random_rotation(11)
        x = icosahedral_grid(L) @ q.T
        n = len(x)
        return dict(name=name, x=x, zeta=rossby_haurwitz(x, 3),
                    area=uniform_areas(n), subset=np.arange(n),
                    theta=0.7, degree=6, seed=11)
    raise KeyError(name)
