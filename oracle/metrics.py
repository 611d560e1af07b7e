"""O4: error measures.  TEST INFRASTRUCTURE ONLY.

* E   -- area-weighted relative l2 velocity error between fast and direct
         summation (Sec. 4, runtime results).
* E_N -- area-weighted relative l2 vorticity error against the exact
         solution (Sec. 4, Rossby-Haurwitz wave); E_inf is its l-infinity
         analogue.
Over a subset of particles the sums run over that subset.
"""

import numpy as np


def rel_l2_velocity(v_fast, v_direct, area):
    v_fast = np.asarray(v_fast, dtype=np.float64)
    v_direct = np.asarray(v_direct, dtype=np.float64)
    a = np.asarray(area, dtype=np.float64)
    num = (((v_fast - v_direct) ** 2).sum(1) * a).sum()
    den = ((v_direct ** 2).sum(1) * a).sum()
    return float(np.sqrt(num / den))


def rel_l2_scalar(z, z_exact, area):
    z = np.asarray(z, dtype=np.float64)
    ze = np.asarray(z_exact, dtype=np.float64)
    a = np.asarray(area, dtype=np.float64)
    return float(np.sqrt((((z - ze) ** 2) * a).sum() / ((ze ** 2) * a).sum()))


def rel_linf_scalar(z, z_exact):
    z = np.asarray(z, dtype=np.float64)
    ze = np.asarray(z_exact, dtype=np.float64)
    return float(np.abs(z - ze).max() / np.abs(ze).max())
