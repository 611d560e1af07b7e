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
* ``ssw_l7``   N = 163842 (level 7), node-patch areas, the polar vortex of the
               vortex-collapse experiment (Sec. 4.4) with its wavenumber-1
               vorticity forcing; time in days; d = 6, theta = 0.7.

``make_ensemble`` builds the ensemble workload: members with seeds 4 + m, each
an icosahedral grid of level 5, 6 or 7 (N = 10242, 40962, 163842) under a
random rotation, node-patch areas, a Rossby-Haurwitz wave of wavenumber 3, 4
or 5 plus a Gaussian bump 1e-6 exp(-(d/0.1)^2) s^-1 at a random centre; RK4
with dt = 1800 s for 24 steps.
"""

import numpy as np

from .grids import (icosahedral_grid, uniform_areas, node_patch_areas,
                    subset_indices, random_rotation)
from .fields import rossby_haurwitz, gaussian_vortex, gaussian_pair, great_circle_distance, polar_vortex

WORKLOADS = ("rh4_l5", "gv_l8", "rh4_l7", "gvpair_l9", "ssw_l7")


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
    if name == "ssw_l7":
        # polar-vortex collapse (Sec. 4.4): the vortex profile on a level-7
        # grid with node-patch areas, time in days (Omega = 2 pi per day),
        # wavenumber-1 forcing with T_p = 4, T_f = 15, lat1 = pi/3; the
        # paper's d = 6, theta = 0.7; dt = 0.01 days (the time step the paper
        # states for its Gaussian-vortex runs; none is given for this one)
        L = 7 if level is None else level
        x, faces = icosahedral_grid(L, return_faces=True)
        return dict(name=name, x=x, zeta=polar_vortex(x), area=node_patch_areas(x, faces),
                    subset=subset_indices(len(x), 4096, 6), theta=0.7, degree=6, seed=6,
                    omega=2.0 * np.pi, dt=0.01, steps=10,
                    forcing=dict(k=1, lat1=np.pi / 3.0, t_ramp=4.0, t_total=15.0))
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


_GRID_CACHE = {}


def _grid_with_areas(level):
    if level not in _GRID_CACHE:
        x, faces = icosahedral_grid(level, return_faces=True)
        _GRID_CACHE[level] = (x, node_patch_areas(x, faces))
    return _GRID_CACHE[level]


def make_member(m, seed0=4, levels=(5, 6, 7)):
    """Member m of the ensemble workload (see the module docstring)."""
    seed = seed0 + m
    rng = np.random.Generator(np.random.PCG64(seed))
    level = int(rng.choice(levels))
    n_wave = int(rng.integers(3, 6))
    c = rng.standard_normal(3)
    c /= np.linalg.norm(c)
    x0, a = _grid_with_areas(level)
    x = x0 @ random_rotation(seed).T
    z = rossby_haurwitz(x, n_wave) + 1e-6 * np.exp(-(great_circle_distance(x, c) / 0.1) ** 2)
    return dict(x=x, zeta=z, area=a.copy(), level=level, n_wave=n_wave, seed=seed)


def make_ensemble(members=48, seed0=4, levels=(5, 6, 7)):
    """Concatenated ensemble: x (N,3), zeta, area (N,), offsets (members+1,)
    and the per-member records."""
    mem = [make_member(m, seed0, levels) for m in range(members)]
    off = np.zeros(members + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(r["x"]) for r in mem])
    return dict(x=np.concatenate([r["x"] for r in mem]), zeta=np.concatenate([r["zeta"] for r in mem]),
                area=np.concatenate([r["area"] for r in mem]), offsets=off, members=mem,
                dt=1800.0, steps=24)


def make_gate_training_input(k, level=7, seed0=100):
    """Training input k of the learned form: an icosahedral grid of the given
    level under a random rotation, A = 4 pi / N, a Rossby-Haurwitz wave of
    wavenumber 3, 4 or 5 plus one to three Gaussian vortices (width 0.1) of
    amplitude +-(0.5..1.5) x 4 pi per day at random centres (seed seed0 + k)."""
    seed = seed0 + k
    rng = np.random.Generator(np.random.PCG64(seed))
    x = icosahedral_grid(level) @ random_rotation(seed).T
    z = rossby_haurwitz(x, int(rng.integers(3, 6)))
    zv = 4.0 * np.pi / 86400.0
    for _ in range(int(rng.integers(1, 4))):
        c = rng.standard_normal(3)
        c /= np.linalg.norm(c)
        amp = zv * rng.uniform(0.5, 1.5) * (1 if rng.uniform() < 0.5 else -1)
        z = z + amp * np.exp(-(great_circle_distance(x, c) / 0.1) ** 2)
    return x, z, uniform_areas(len(x))
