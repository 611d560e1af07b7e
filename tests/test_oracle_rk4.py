"""Pins for the oracle RK4 stepper (O3): fourth-order convergence on a velocity
field with a closed-form flow, the vorticity invariant of the BVE, and the
Rossby-Haurwitz phase speed."""

import numpy as np
import pytest

import synthetic as S
from oracle import direct, rk4


def _solid_body(omega):
    ez = np.array([0.0, 0.0, 1.0])

    def vel(x, zeta, area):
        return omega * np.cross(ez[None, :], x)
    return vel


def test_rk4_fourth_order_on_solid_body_rotation():
    """u = omega z_hat x x rotates the sphere rigidly: x(t) = Rz(omega t) x0."""
    x0 = S.random_sphere_points(50, 0)
    om = 1.3
    T_end = 1.0
    errs = []
    for nsteps in (8, 16, 32):
        x, z = rk4.integrate(x0, np.zeros(50), np.ones(50), T_end / nsteps, 0.0, nsteps,
                             _solid_body(om))
        c, s = np.cos(om * T_end), np.sin(om * T_end)
        R = np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])
        errs.append(np.abs(x - x0 @ R.T).max())
    for e0, e1 in zip(errs, errs[1:]):
        assert 12 < e0 / e1 < 20, errs


def test_vorticity_tracks_height():
    """d zeta / dt = -2 Omega dz/dt and RK4 is linear in its stage slopes, so
    zeta(t) - zeta(0) = -2 Omega (z(t) - z(0)) up to rounding.  The sphere
    projection after each step moves z (not zeta) by the RK4 truncation
    error, so the invariant is checked with the projection switched off."""
    x0 = S.icosahedral_grid(2)
    n = len(x0)
    z0 = S.rossby_haurwitz(x0, 4)
    a = S.uniform_areas(n)
    Om = S.OMEGA_EARTH_S
    vel = lambda x, zz, aa: direct.velocity(x, zz, aa)
    x, z = rk4.integrate(x0, z0, a, 1800.0, Om, 4, vel, project=False)
    drift = (z - z0) + 2 * Om * (x[:, 2] - x0[:, 2])
    assert np.abs(drift).max() < 1e-12 * np.abs(z0).max() + 1e-16


@pytest.mark.slow
def test_rh_wave_phase_speed():
    """Sec. 4: the RH wave of wavenumber n moves east at
    nu = (n(3+n) w - 2 Omega) / ((1+n)(2+n)).  With n = 4 and
    w = K = 7.848e-6 s^-1, integrate 12 h and compare the wave's longitude
    shift (phase of sum A zeta Y_5^4-projection) with nu * t."""
    L = 4
    x0, f = S.icosahedral_grid(L, return_faces=True)
    a = S.node_patch_areas(x0, f)
    n, w = 4, 7.848e-6
    Om = S.OMEGA_EARTH_S
    z0 = S.rossby_haurwitz(x0, n, omega=w, K=w)
    vel = lambda x, zz, aa: direct.velocity(x, zz, aa)
    dt, steps = 3600.0, 12
    x, z = rk4.integrate(x0, z0, a, dt, Om, steps, vel)

    def phase(x, zz):
        c = ((x[:, 0] + 1j * x[:, 1]) ** n * x[:, 2] * zz * a).sum()
        return np.angle(c)
    # zeta's wave part is -K(n+1)(n+2) z Re((x+iy)^n); shifted east by delta
    # its projection on conj((x+iy)^n) z turns by n * delta
    dphi = np.angle(np.exp(1j * (phase(x, z) - phase(x0, z0)))) / n
    nu = (n * (3 + n) * w - 2 * Om) / ((1 + n) * (2 + n))
    expected = nu * dt * steps
    assert abs(dphi - expected) < 0.05 * abs(expected) + 2e-3, (dphi, expected)
