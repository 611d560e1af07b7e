"""Pins for the oracle's error measures (O4; Sec. 4, runtime results and
Rossby-Haurwitz wave): the area-weighted relative l2 norms on hand-computed
cases with unequal areas, where the unweighted norm gives a different value."""

import numpy as np

from oracle import metrics


def test_velocity_error_is_area_weighted():
    # E = sqrt(sum_i A_i |u_i - v_i|^2 / sum_i A_i |v_i|^2)
    # rows: |u - v|^2 = 0, 0.01, 0.04; |v|^2 = 1, 1, 4; A = 1, 3, 0.5
    v = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 2.0]])
    u = np.array([[1.0, 0.0, 0.0], [0.0, 1.1, 0.0], [0.0, 0.2, 2.0]])
    a = np.array([1.0, 3.0, 0.5])
    want = np.sqrt((3.0 * 0.01 + 0.5 * 0.04) / (1.0 + 3.0 + 0.5 * 4.0))   # sqrt(0.05 / 6) = 0.0912871
    assert abs(metrics.rel_l2_velocity(u, v, a) - want) < 1e-15
    assert abs(want - 0.09128709291752768) < 1e-15
    # equal areas give the plain relative l2 norm sqrt(0.05 / 6) = 0.0913 here;
    # other weights move it: A = 2, 1, 1 gives sqrt((0.01 + 0.04) / 7) = 0.0845
    assert abs(metrics.rel_l2_velocity(u, v, np.ones(3)) - np.sqrt(0.05 / 6.0)) < 1e-15
    a2 = np.array([2.0, 1.0, 1.0])
    assert abs(metrics.rel_l2_velocity(u, v, a2) - np.sqrt(0.05 / 7.0)) < 1e-15
    a3 = np.array([1.0, 1.0, 4.0])
    want3 = np.sqrt((0.01 + 4.0 * 0.04) / (1.0 + 1.0 + 16.0))
    assert abs(metrics.rel_l2_velocity(u, v, a3) - want3) < 1e-15


def test_vorticity_error_is_area_weighted():
    # E_N = sqrt(sum_i A_i (z_i - e_i)^2 / sum_i A_i e_i^2) over the particles
    e = np.array([2.0, -1.0, 0.5, 0.0])
    z = np.array([2.5, -1.0, 0.5, 0.1])
    a = np.array([0.25, 2.0, 4.0, 1.0])
    # numerator 0.25 * 0.25 + 1.0 * 0.01 = 0.0725; denominator 0.25 * 4 + 2 + 4 * 0.25 = 4
    assert abs(metrics.rel_l2_scalar(z, e, a) - np.sqrt(0.0725 / 4.0)) < 1e-15
    # the same errors with equal areas: sqrt(0.26 / 5.25)
    assert abs(metrics.rel_l2_scalar(z, e, np.ones(4)) - np.sqrt(0.26 / 5.25)) < 1e-15
    assert abs(metrics.rel_linf_scalar(z, e) - 0.25) < 1e-15
