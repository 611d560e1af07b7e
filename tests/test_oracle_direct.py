"""Pins for the oracle's direct sum (O1) against what the mathematics fixes:
brute force in 50-digit arithmetic, invariants, and the closed-form
Rossby-Haurwitz velocity."""

import json
import os

import mpmath
import numpy as np
import pytest

import synthetic as S
from oracle import direct, metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def _brute_force_mp(x, zeta, area, dps=50):
    """Literal discrete BVE sum (Sec. 2) in 50-digit arithmetic, pair by pair."""
    mpmath.mp.dps = dps
    n = len(x)
    X = [[mpmath.mpf(float(c)) for c in row] for row in x]
    q = [mpmath.mpf(float(zeta[j])) * mpmath.mpf(float(area[j])) for j in range(n)]
    out = np.zeros((n, 3))
    for i in range(n):
        acc = [mpmath.mpf(0)] * 3
        xi = X[i]
        for j in range(n):
            if j == i:
                continue
            xj = X[j]
            cross = [xi[1] * xj[2] - xi[2] * xj[1], xi[2] * xj[0] - xi[0] * xj[2],
                     xi[0] * xj[1] - xi[1] * xj[0]]
            den = 1 - (xi[0] * xj[0] + xi[1] * xj[1] + xi[2] * xj[2])
            for c in range(3):
                acc[c] += cross[c] * q[j] / den
        for c in range(3):
            out[i, c] = float(-acc[c] / (4 * mpmath.pi))
    return out


@pytest.mark.parametrize("level,rot", [(0, None), (1, None), (1, 7)])
def test_direct_matches_50_digit_brute_force(level, rot):
    x = S.icosahedral_grid(level)
    if rot is not None:
        x = x @ S.random_rotation(rot).T
    n = len(x)
    rng = np.random.default_rng(level + 1)
    zeta = rng.standard_normal(n)
    area = S.uniform_areas(n) * (1 + 0.1 * rng.random(n))
    ref = _brute_force_mp(x, zeta, area)
    for den in ("dot", "dist2"):
        u = direct.velocity(x, zeta, area, den=den)
        err = np.abs(u - ref).max() / np.abs(ref).max()
        assert err < 1e-13, (den, err)


def test_direct_subset_equals_full_rows():
    x = S.random_sphere_points(700, 3)
    z = np.random.default_rng(0).standard_normal(700)
    a = S.uniform_areas(700)
    full = direct.velocity(x, z, a)
    idx = np.array([0, 5, 699, 350])
    sub = direct.velocity(x, z, a, targets=idx)
    np.testing.assert_array_equal(sub, full[idx])


def test_tangency_rotation_linearity():
    x = S.icosahedral_grid(3)
    n = len(x)
    z = S.rossby_haurwitz(x, 4)
    a = S.uniform_areas(n)
    u = direct.velocity(x, z, a)
    # tangency x_i . u_i = 0
    tang = np.abs((x * u).sum(1)).max() / np.abs(u).max()
    assert tang < 1e-15
    # rotation equivariance u(Qx) = Q u(x)
    Q = S.random_rotation(5)
    uq = direct.velocity(x @ Q.T, z, a)
    assert np.abs(uq - u @ Q.T).max() / np.abs(u).max() < 1e-13
    # linearity in the charges
    z2 = np.random.default_rng(1).standard_normal(n)
    u2 = direct.velocity(x, z2, a)
    u12 = direct.velocity(x, 2.0 * z - 3.0 * z2, a)
    assert np.abs(u12 - (2.0 * u - 3.0 * u2)).max() / np.abs(u12).max() < 1e-13
    # the two denominators agree on the sphere (Sec. 2, alternative kernel)
    ud = direct.velocity(x, z, a, den="dist2")
    assert np.abs(ud - u).max() / np.abs(u).max() < 1e-13


def rh_exact_velocity(x, n, omega, K):
    """u = x x grad(psi) with psi = -omega z + K z Re((x+iy)^n), the stream
    function of the RH vorticity (Laplacian eigenfunctions of degree 1 and
    n + 1: eigenvalues -2 and -(n+1)(n+2))."""
    w1 = (x[:, 0] + 1j * x[:, 1]) ** (n - 1)
    wn = (x[:, 0] + 1j * x[:, 1]) ** n
    z = x[:, 2]
    g = np.stack([K * n * z * w1.real, -K * n * z * w1.imag, -omega + K * wn.real], 1)
    return np.cross(x, g)


def test_rh_closed_form_convergence():
    """With node-patch areas the midpoint-rule sum converges to the exact RH
    velocity at second order (the error drops ~4x per refinement)."""
    errs = []
    for L in (3, 4, 5):
        x, f = S.icosahedral_grid(L, return_faces=True)
        a = S.node_patch_areas(x, f)
        z = S.rossby_haurwitz(x, 4, omega=1.0, K=1.0)
        u = direct.velocity(x, z, a)
        ue = rh_exact_velocity(x, 4, 1.0, 1.0)
        errs.append(metrics.rel_l2_velocity(u, ue, a))
    assert errs[0] < 0.05
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.0 < e0 / e1 < 5.0, errs


def test_solid_body_rotation():
    """zeta = 2 omega z is solid-body rotation u = omega z_hat x x."""
    x, f = S.icosahedral_grid(5, return_faces=True)
    a = S.node_patch_areas(x, f)
    u = direct.velocity(x, 2.0 * x[:, 2], a)
    ue = np.cross(np.array([0.0, 0.0, 1.0])[None, :], x)
    assert metrics.rel_l2_velocity(u, ue, a) < 2e-3


def test_rh_paper_form_matches_printed_coefficients():
    g = json.load(open(GOLDEN))["rh_stationary_k4"]
    x = S.random_sphere_points(50, 0)
    lat = np.arcsin(x[:, 2])
    lon = np.arctan2(x[:, 1], x[:, 0])
    printed = g["two_w"] * np.sin(lat) + g["amplitude"] * np.sin(lat) * np.cos(lat) ** 4 * np.cos(4 * lon)
    np.testing.assert_allclose(S.rossby_haurwitz_paper(x, 4), printed, rtol=1e-12, atol=1e-12)


def test_grid_sizes_match_paper():
    g = json.load(open(GOLDEN))["grid_sizes"]
    for lvl, n in g.items():
        if lvl.startswith("_"):
            continue
        assert S.grid_size(int(lvl)) == n
    assert len(S.icosahedral_grid(3)) == 642
