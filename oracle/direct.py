"""O1: the direct O(N^2) velocity sum -- the exact result the tree code
approximates.  TEST INFRASTRUCTURE ONLY (see the package docstring).

Discrete BVE system (Sec. 2, midpoint rule of the Biot-Savart integral):

    u_i = -(1 / 4 pi) * sum_{j != i} (x_i x x_j) zeta_j A_j / (1 - x_i . x_j)

The denominator is either the literal 1 - x_i . x_j ("dot") or the
alternative |x_i - x_j|^2 / 2 ("dist2"), equal on the unit sphere (Sec. 2,
alternative kernel equation).  The self term j = i is excluded by index.
Every pair's cross product is formed and summed as written; nothing is
factored out.  The only library step is NumPy elementwise arithmetic.
"""

import numpy as np

FOUR_PI = 4.0 * np.pi


def _den(xt, xs, den):
    if den == "dot":
        dot = (xt[:, None, 0] * xs[None, :, 0] + xt[:, None, 1] * xs[None, :, 1]) \
            + xt[:, None, 2] * xs[None, :, 2]
        return 1.0 - dot
    if den == "dist2":
        d0 = xt[:, None, 0] - xs[None, :, 0]
        d1 = xt[:, None, 1] - xs[None, :, 1]
        d2 = xt[:, None, 2] - xs[None, :, 2]
        return 0.5 * ((d0 * d0 + d1 * d1) + d2 * d2)
    raise ValueError(den)


def velocity(x, zeta, area, targets=None, den="dot", chunk_elems=1 << 22):
    """Velocity u_i (len(targets), 3) of the discrete BVE system.

    x: (N, 3) particles on the unit sphere; zeta, area: (N,); targets: indices
    of the particles to evaluate (default all).  Sources are all N particles.
    """
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(zeta, dtype=np.float64) * np.asarray(area, dtype=np.float64)
    n = len(x)
    targets = np.arange(n) if targets is None else np.asarray(targets)
    out = np.empty((len(targets), 3))
    m = max(1, chunk_elems // max(n, 1))
    for c0 in range(0, len(targets), m):
        idx = targets[c0:c0 + m]
        xt = x[idx]
        dn = _den(xt, x, den)
        w = q[None, :] / np.where(idx[:, None] == np.arange(n)[None, :], np.inf, dn)
        # (x_i x x_j) for every pair, then sum_j of w_ij (x_i x x_j)
        cx = xt[:, None, 1] * x[None, :, 2] - xt[:, None, 2] * x[None, :, 1]
        cy = xt[:, None, 2] * x[None, :, 0] - xt[:, None, 0] * x[None, :, 2]
        cz = xt[:, None, 0] * x[None, :, 1] - xt[:, None, 1] * x[None, :, 0]
        out[c0:c0 + m, 0] = (w * cx).sum(1)
        out[c0:c0 + m, 1] = (w * cy).sum(1)
        out[c0:c0 + m, 2] = (w * cz).sum(1)
    return -out / FOUR_PI


def kernel_sum(xt, xs, q, kernel, exclude=None):
    """sum_j q_j K(xt_i, xs_j) for a generic vector kernel K(X, Y) -> (a, b, 3).

    `exclude` (optional (a,) int array): for target i skip source exclude[i].
    Used to compare the tree code with a direct sum for any kernel."""
    k = kernel(xt, xs)
    w = np.broadcast_to(q[None, :], k.shape[:2]).copy()
    if exclude is not None:
        rows = np.arange(len(xt))
        ok = exclude >= 0
        w[rows[ok], exclude[ok]] = 0.0
    return (w[:, :, None] * k).sum(1)


def stream_function(x, zeta, area, targets=None, den="dot", chunk_elems=1 << 22):
    """Stream function psi_i (len(targets),) of the discrete system:

        psi_i = (1 / 4 pi) * sum_{j != i} zeta_j A_j log(1 - x_i . x_j)

    the midpoint rule of psi = int G zeta with the Green's function of the
    Laplace-Beltrami operator on the unit sphere (Sec. 2, stream function and
    Green's function).  Reading: the sign is the one for which Delta psi = zeta
    (zero-mean zeta) and u = x x grad psi reproduce the Biot-Savart velocity
    above; the paper's G carries the opposite sign (see the velocity's sign
    reading).  `den` selects 1 - x.y or |x - y|^2 / 2 inside the logarithm."""
    x = np.asarray(x, dtype=np.float64)
    q = np.asarray(zeta, dtype=np.float64) * np.asarray(area, dtype=np.float64)
    n = len(x)
    targets = np.arange(n) if targets is None else np.asarray(targets)
    out = np.empty(len(targets))
    m = max(1, chunk_elems // max(n, 1))
    for c0 in range(0, len(targets), m):
        idx = targets[c0:c0 + m]
        dn = _den(x[idx], x, den)
        self_pair = idx[:, None] == np.arange(n)[None, :]
        lg = np.log(np.where(self_pair, 1.0, dn))
        out[c0:c0 + m] = (np.where(self_pair, 0.0, q[None, :] * lg)).sum(1)
    return out / FOUR_PI
