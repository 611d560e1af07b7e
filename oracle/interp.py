"""Interpolation in spherical triangles.  TEST INFRASTRUCTURE ONLY.

Sec. 3 (interpolation in triangles): a point v of a spherical triangle
(v1, v2, v3) is written v = b1 v1 + b2 v2 + b3 v3, b >= 0 (spherical
barycentric coordinates, i.e. b = M^{-1} v with M = [v1 v2 v3]), and the
spherical Bernstein-Bezier basis of degree d is b1^i b2^j b3^k, i + j + k = d,
(d+1)(d+2)/2 functions.

Readings (the paper names approximate Fekete points but does not give them):

* Basis scaling: the multinomial d! / (i! j! k!) multiplies each basis
  function.  It spans the same space and only improves conditioning.
* Points: the Lobatto triangle grid of Blyth & Pozrikidis (2006): with
  v_0..v_d the Gauss-Lobatto-Legendre nodes on [0, 1], point (i, j, k) has
  planar barycentrics ((1 + 2 v_i - v_j - v_k) / 3, (1 + 2 v_j - v_i - v_k) / 3,
  (1 + 2 v_k - v_i - v_j) / 3); on a spherical triangle it is mapped to
  normalise(b1 v1 + b2 v2 + b3 v3).
* Enumeration of (i, j, k), shared by points and basis: i = 0..d, then
  j = 0..d-i, k = d - i - j.
"""

from math import factorial

import numpy as np


def n_basis(d):
    return (d + 1) * (d + 2) // 2


def multi_indices(d):
    return [(i, j, d - i - j) for i in range(d + 1) for j in range(d - i + 1)]


def gll_nodes01(d):
    """Gauss-Lobatto-Legendre nodes on [0, 1]: the endpoints and the roots of
    the derivative of the Legendre polynomial P_d (mapped from [-1, 1])."""
    if d == 0:
        return np.array([0.5])
    if d == 1:
        return np.array([0.0, 1.0])
    inner = np.polynomial.legendre.Legendre.basis(d).deriv().roots()
    inner = np.sort(inner.real)
    # polish each root with Newton steps on P_d'
    dp = np.polynomial.legendre.Legendre.basis(d).deriv()
    ddp = dp.deriv()
    for _ in range(3):
        inner = inner - dp(inner) / ddp(inner)
    t = np.concatenate([[-1.0], inner, [1.0]])
    return 0.5 * (1.0 + t)


def reference_points(d):
    """Planar barycentrics (n_p, 3) of the interpolation points."""
    v = gll_nodes01(d)
    pts = []
    for i, j, k in multi_indices(d):
        pts.append(((1 + 2 * v[i] - v[j] - v[k]) / 3.0,
                    (1 + 2 * v[j] - v[i] - v[k]) / 3.0,
                    (1 + 2 * v[k] - v[i] - v[j]) / 3.0))
    return np.array(pts)


def basis(beta, d):
    """Scaled SBB basis at barycentrics beta (M, 3) -> (M, n_p)."""
    beta = np.atleast_2d(beta)
    out = np.empty((len(beta), n_basis(d)))
    fd = factorial(d)
    for col, (i, j, k) in enumerate(multi_indices(d)):
        c = fd // (factorial(i) * factorial(j) * factorial(k))
        out[:, col] = c * beta[:, 0] ** i * beta[:, 1] ** j * beta[:, 2] ** k
    return out


def proxy_points(tri, d):
    """Interpolation points of one spherical triangle tri (3, 3)."""
    b = reference_points(d)
    p = (b[:, 0:1] * tri[0][None, :] + b[:, 1:2] * tri[1][None, :]) + b[:, 2:3] * tri[2][None, :]
    n = np.sqrt((p * p).sum(1))
    return p / n[:, None]


def barycentric(tri, y):
    """Spherical barycentric coordinates b = M^{-1} y, M = [v1 v2 v3]."""
    m = np.stack([tri[0], tri[1], tri[2]], axis=1)
    return np.linalg.solve(m, np.atleast_2d(y).T).T


def lagrange_matrix(tri, d, y):
    """L[i, m] = L_m(y_i): the Lagrange basis of the triangle's interpolation
    points, L_m(y) = sum_k (V^{-1})_{km} B_k(y) with V_{mk} = B_k(proxy_m)."""
    prox = proxy_points(tri, d)
    V = basis(barycentric(tri, prox), d)
    Vinv = np.linalg.inv(V)
    return basis(barycentric(tri, y), d) @ Vinv


def lebesgue_sample(d, samples=2000, seed=0):
    """Sampled Lebesgue constant of the reference points on the planar
    triangle (diagnostic for the choice of points)."""
    rng = np.random.default_rng(seed)
    b = rng.dirichlet([1, 1, 1], size=samples)
    V = basis(reference_points(d), d)
    L = basis(b, d) @ np.linalg.inv(V)
    return float(np.abs(L).sum(1).max())
