"""Pins for the oracle's stream function (Sec. 2, stream function and Green's
function): 50-digit brute force on tiny sets, the closed-form Rossby-Haurwitz stream function, u = x x grad(psi)
against the (separately pinned) Biot-Savart velocity, and the tree code's
reduction to the direct sum."""

from decimal import Decimal, getcontext

import numpy as np
import pytest

import synthetic as S
from oracle import direct, tree

PI50 = Decimal("3.14159265358979323846264338327950288419716939937510582097494")


def _brute(x, q, den):
    getcontext().prec = 50
    X = [[Decimal(float(v)) for v in row] for row in x]
    Q = [Decimal(float(v)) for v in q]
    out = []
    for i in range(len(X)):
        acc = Decimal(0)
        for j in range(len(X)):
            if j == i:
                continue
            if den == "dot":
                d = 1 - (X[i][0] * X[j][0] + X[i][1] * X[j][1] + X[i][2] * X[j][2])
            else:
                d = sum((X[i][k] - X[j][k]) ** 2 for k in range(3)) / 2
            acc += Q[j] * d.ln()
        out.append(float(acc / (4 * PI50)))
    return np.array(out)


@pytest.mark.parametrize("den", ["dot", "dist2"])
@pytest.mark.parametrize("level,rot", [(0, None), (1, 3)])
def test_brute_force_50_digits(den, level, rot):
    x = S.icosahedral_grid(level)
    if rot is not None:
        x = x @ S.random_rotation(rot).T
    rng = np.random.default_rng(level + 7)
    z = rng.uniform(-1.0, 1.0, len(x))
    a = rng.uniform(0.5, 1.5, len(x))
    got = direct.stream_function(x, z, a, den=den)
    want = _brute(x, z * a, den)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def _rh_stream(x, n, omega, K):
    """Closed form: zeta = 2 w sin(phi) - K (n+1)(n+2) cos^n(phi) sin(phi) cos(n lam)
    is a sum of spherical harmonics of degrees 1 and n + 1 (eigenvalues -2 and
    -(n+1)(n+2) of the Laplace-Beltrami operator), so the zero-mean solution of
    Delta psi = zeta is psi = -w sin(phi) + K cos^n(phi) sin(phi) cos(n lam)."""
    re = ((x[:, 0] + 1j * x[:, 1]) ** n).real
    return -omega * x[:, 2] + K * x[:, 2] * re


def test_rossby_haurwitz_closed_form_convergence():
    """The midpoint rule with node-patch areas converges to the closed form at
    second order (errors fall by about 4x per refinement)."""
    errs = []
    for level in (3, 4, 5):
        x, faces = S.icosahedral_grid(level, return_faces=True)
        a = S.node_patch_areas(x, faces)
        z = S.rossby_haurwitz(x, 4, 1.0, 1.0)
        psi = direct.stream_function(x, z, a)
        ex = _rh_stream(x, 4, 1.0, 1.0)
        errs.append(np.sqrt(((psi - ex) ** 2 * a).sum() / ((ex ** 2) * a).sum()))
    assert errs[-1] < 1e-2, errs
    for e0, e1 in zip(errs, errs[1:]):
        assert 2.5 < e0 / e1 < 6.0, errs


def test_velocity_is_x_cross_grad_psi():
    """u = x x grad(psi): differences of psi at a point with zero charge,
    crossed with the point, give the Biot-Savart velocity there (this ties the
    stream function's sign and factor to the velocity's pins)."""
    xs = S.random_sphere_points(300, 4)
    rng = np.random.default_rng(4)
    z = rng.uniform(-1.0, 1.0, 300)
    p = S.random_sphere_points(1, 44)[0]
    h = 1e-5
    zz = np.concatenate([z, [0.0]])
    a = np.ones(301)

    def psi_at(pt):  # one extra particle of zero charge at pt (off the sphere is fine)
        return direct.stream_function(np.concatenate([xs, [pt]]), zz, a, targets=np.array([300]))[0]

    def cd(e, hh):
        return (psi_at(p + hh * e) - psi_at(p - hh * e)) / (2 * hh)

    # central differences with one Richardson step (error O(h^4))
    grad = np.array([(4.0 * cd(e, h) - cd(e, 2 * h)) / 3.0 for e in np.eye(3)])
    u_psi = np.cross(p, grad)
    u = direct.velocity(np.concatenate([xs, [p]]), zz, a, targets=np.array([300]))[0]
    assert np.abs(u_psi - u).max() <= 1e-7 * np.abs(u).max()


@pytest.mark.parametrize("den", ["dot", "dist2"])
def test_tree_reduces_to_direct_and_approximates_it(den):
    x = S.icosahedral_grid(3) @ S.random_rotation(5).T
    z = S.rossby_haurwitz(x, 3)
    a = S.uniform_areas(len(x))
    ref = direct.stream_function(x, z, a, den=den)
    scale = np.abs(ref).max()
    # theta -> 0: nothing is separated, every pair is a direct (PP) interaction
    t0 = tree.TreeCode(x, z, a, theta=1e-9, degree=4, n_crit=16, den=den, kernel=tree.stream_kernel(den))
    assert np.abs(t0.stream_function() - ref).max() <= 1e-13 * scale
    t1 = tree.TreeCode(x, z, a, theta=0.7, degree=8, n_crit=16, den=den, kernel=tree.stream_kernel(den))
    assert sum(len(v) for k, v in t1.lists.items() if k != "PP") > 0
    err = np.abs(t1.stream_function() - ref).max() / scale
    assert err < 1e-4, err
