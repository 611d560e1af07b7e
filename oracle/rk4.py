"""O3: classical RK4 for the Lagrangian BVE particle system.
TEST INFRASTRUCTURE ONLY.

State (x, zeta); right-hand side (Sec. 2, discrete system)
    dx_i/dt    = u_i(x; zeta A)
    dzeta_i/dt = -2 Omega dz_i/dt = -2 Omega u_i,z
The velocity is re-evaluated from scratch at every stage (the tree is rebuilt
for the stage positions).  Readings: stage positions are used as computed
(the |x - y|^2 / 2 kernel is well defined off the sphere, Sec. 2; with
1 - x . y the denominator of close pairs vanishes there, so time stepping
uses the former); after each full step every particle is projected back to
the unit sphere, x <- x / |x|.  The
areas A are constant in time.
"""

import numpy as np


def rhs(x, zeta, area, omega, velocity_fn):
    u = velocity_fn(x, zeta, area)
    return u, -2.0 * omega * u[:, 2]


def step(x, zeta, area, dt, omega, velocity_fn, project=True):
    k1x, k1z = rhs(x, zeta, area, omega, velocity_fn)
    k2x, k2z = rhs(x + 0.5 * dt * k1x, zeta + 0.5 * dt * k1z, area, omega, velocity_fn)
    k3x, k3z = rhs(x + 0.5 * dt * k2x, zeta + 0.5 * dt * k2z, area, omega, velocity_fn)
    k4x, k4z = rhs(x + dt * k3x, zeta + dt * k3z, area, omega, velocity_fn)
    xn = x + (dt / 6.0) * (k1x + 2.0 * k2x + 2.0 * k3x + k4x)
    zn = zeta + (dt / 6.0) * (k1z + 2.0 * k2z + 2.0 * k3z + k4z)
    if project:
        xn = xn / np.sqrt((xn * xn).sum(1))[:, None]
    return xn, zn


def integrate(x, zeta, area, dt, omega, n_steps, velocity_fn, project=True):
    for _ in range(n_steps):
        x, zeta = step(x, zeta, area, dt, omega, velocity_fn, project)
    return x, zeta
