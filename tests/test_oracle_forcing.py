"""Pins for the oracle's vorticity forcing (O4; Sec. 4.4, polar vortex collapse):
the ramp's values at its breakpoints and its time symmetry, the latitude
profile's maximum at the latitude of maximum forcing, the Rossby number the
paper prints, the zonal structure cos(k lon), linearity of the forced
velocity, and the stage times of the forced RK4 step."""

import json
import os

import numpy as np
import pytest

import synthetic as S
from oracle import direct, forcing, rk4

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))["ssw_forcing"]
TP, TF, LAT1 = GOLD["t_ramp_days"], GOLD["t_total_days"], GOLD["lat1"]
OMEGA = S.OMEGA_EARTH_DAY


def test_ramp_breakpoints_and_time_symmetry():
    """A(0) = 0, A = 1/2 halfway up and halfway down, 1 on the plateau, 0 from
    T_f on; continuous at every breakpoint; and A(t) = A(T_f - t): the
    ramp-down is the ramp-up reversed in time."""
    A = lambda t: forcing.ramp(t, TP, TF)
    assert A(0.0) == 0.0 and A(-1.0) == 0.0 and A(TF) == 0.0 and A(TF + 3.0) == 0.0
    assert A(TP / 2) == pytest.approx(0.5, abs=1e-15)
    assert A(TF - TP / 2) == pytest.approx(0.5, abs=1e-15)
    assert A(TP) == 1.0 and A(0.5 * TF) == 1.0
    eps = 1e-9
    for tb in (0.0, TP, TF - TP, TF):
        assert abs(A(tb - eps) - A(tb + eps)) < 1e-12, tb
    for t in np.linspace(0.0, TF, 301):
        assert A(t) == pytest.approx(A(TF - t), abs=1e-14), t
    ts = np.linspace(0.0, TP, 101)
    assert np.all(np.diff([A(t) for t in ts]) > 0.0)


def test_latitude_profile_peaks_at_lat1_with_value_one():
    """B = s e^(1 - s) with s = tan^2(lat1) / tan^2(lat): s e^(1-s) <= 1 with
    equality only at s = 1, i.e. at lat = lat1; zero south of the equator and
    vanishing towards the equator and the pole."""
    lat = np.linspace(-np.pi / 2, np.pi / 2, 200001)
    b = forcing.latitude_profile(lat, LAT1)
    assert b.max() <= 1.0 + 1e-15
    assert lat[np.argmax(b)] == pytest.approx(LAT1, abs=2e-5)
    assert forcing.latitude_profile(np.array([LAT1]), LAT1)[0] == pytest.approx(1.0, abs=1e-15)
    assert np.all(b[lat <= 0.0] == 0.0)
    assert forcing.latitude_profile(np.array([1e-3, np.pi / 2 - 1e-9]), LAT1).max() < 1e-6


@pytest.mark.parametrize("k", GOLD["wavenumbers"])
def test_rossby_number_is_point_three_k_squared(k):
    """The paper gives the forcing's Rossby number as 0.3 k^2: max |F_R| over
    the sphere, at full ramp, divided by 2 Omega."""
    lat = np.linspace(0.0, np.pi / 2, 4001)[1:-1]
    lon = np.linspace(-np.pi, np.pi, 721)
    LA, LO = np.meshgrid(lat, lon, indexing="ij")
    x = np.stack([np.cos(LA) * np.cos(LO), np.cos(LA) * np.sin(LO), np.sin(LA)], -1).reshape(-1, 3)
    f = forcing.forcing(x, 0.5 * TF, k, OMEGA, LAT1, TP, TF)
    ro = np.abs(f).max() / (2.0 * OMEGA)
    assert ro == pytest.approx(GOLD["rossby_number_per_k2"] * k * k, rel=1e-6)


@pytest.mark.parametrize("k", [1, 2, 3])
def test_zonal_structure(k):
    """cos(k lon): periodic in 2 pi / k, odd under a half period, zero zonal
    mean on equally spaced longitudes, positive at lon = 0; and the same
    value anywhere along a ray from the origin (stage points off the sphere)."""
    lat = 0.8
    lon = np.linspace(0.0, 2 * np.pi, 64, endpoint=False) + 0.1
    pt = lambda lo: np.stack([np.cos(lat) * np.cos(lo), np.cos(lat) * np.sin(lo), np.full_like(lo, np.sin(lat))], -1)
    f = lambda lo: forcing.forcing(pt(lo), 5.0, k, OMEGA, LAT1, TP, TF)
    assert np.allclose(f(lon + 2 * np.pi / k), f(lon), atol=1e-12)
    assert np.allclose(f(lon + np.pi / k), -f(lon), atol=1e-12)
    assert abs(f(lon).mean()) < 1e-12
    assert f(np.array([0.0]))[0] > 0.0
    assert np.allclose(forcing.forcing(1.7 * pt(lon), 5.0, k, OMEGA, LAT1, TP, TF), f(lon), rtol=1e-13, atol=0)


def test_forced_velocity_is_linear_in_the_forcing():
    """The Biot-Savart sum is linear in the charges: the forced velocity is the
    unforced one minus the velocity induced by F_R alone."""
    x = S.icosahedral_grid(3)
    a = S.uniform_areas(len(x))
    z = S.polar_vortex(x)
    t = 6.0
    fz = forcing.forced_zeta(x, z, t, 2, OMEGA, LAT1, TP, TF)
    fr = forcing.forcing(x, t, 2, OMEGA, LAT1, TP, TF)
    u = direct.velocity(x, fz, a)
    assert np.allclose(u, direct.velocity(x, z, a) - direct.velocity(x, fr, a), rtol=0, atol=1e-12 * np.abs(u).max())
    assert np.abs(fr).max() > 0.1


def test_forced_step_sees_the_rk4_stage_times():
    """With a velocity that ignores its input the particles stand still, so the
    field handed to the velocity at each stage is zeta - F_R(x, t + c dt) with
    the classical RK4 nodes c = 0, 1/2, 1/2, 1."""
    x = S.random_sphere_points(40, 3)
    x[:, 2] = np.abs(x[:, 2])  # northern hemisphere: F_R != 0
    z = np.linspace(-1.0, 1.0, 40)
    seen = []

    def vel(xs, zs, area):
        seen.append(zs.copy())
        return np.zeros_like(xs)

    t0, dt = 0.7, 0.4
    xn, zn = forcing.rk4_step(x, z, np.ones(40), t0, dt, OMEGA, vel, (1, LAT1, TP, TF))
    assert np.array_equal(zn, z) and np.allclose(xn, x, atol=1e-15)
    for got, c in zip(seen, (0.0, 0.5, 0.5, 1.0)):
        want = z - forcing.forcing(x, t0 + c * dt, 1, OMEGA, LAT1, TP, TF)
        assert np.array_equal(got, want)
    assert not np.array_equal(seen[0], seen[3])


def test_forced_step_after_the_forcing_ends_is_the_plain_step():
    """From T_f on A = 0, so the forced step equals the oracle's plain step."""
    x = S.icosahedral_grid(2)
    a = S.uniform_areas(len(x))
    z = S.polar_vortex(x)
    vel = lambda xs, zs, ar: direct.velocity(xs, zs, ar, den="dist2")
    x1, z1 = forcing.rk4_step(x, z, a, TF + 1.0, 0.01, OMEGA, vel, (2, LAT1, TP, TF))
    x2, z2 = rk4.step(x, z, a, 0.01, OMEGA, vel)
    assert np.array_equal(x1, x2) and np.array_equal(z1, z2)
