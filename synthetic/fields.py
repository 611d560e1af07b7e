"""Initial vorticity fields of the paper's test cases (Sec. 4) and the seeded
variants the benchmarks use.  All functions take Cartesian points on the unit
sphere, shape (N, 3), and return FP64 arrays.

Latitude phi = asin(z), longitude lambda = atan2(y, x); in Cartesian form
sin(phi) = z and cos(phi)^n cos(n lambda) = Re((x + i y)^n).
"""

import numpy as np

#: Earth's rotation rate, 2 pi per day (Sec. 2), in s^-1 and in day^-1.
OMEGA_EARTH_S = 2.0 * np.pi / 86400.0
OMEGA_EARTH_DAY = 2.0 * np.pi


def lonlat(x):
    lat = np.arcsin(np.clip(x[:, 2], -1.0, 1.0))
    lon = np.arctan2(x[:, 1], x[:, 0])
    return lon, lat


def _re_im_pow(x, n):
    w = (x[:, 0] + 1j * x[:, 1]) ** n
    return w.real, w.imag


def rossby_haurwitz(x, n=4, omega=7.848e-6, K=7.848e-6):
    """Williamson-style Rossby-Haurwitz wave, wavenumber n:
    zeta = 2 omega sin(phi) - K (n+1)(n+2) cos^n(phi) sin(phi) cos(n lambda)."""
    re, _ = _re_im_pow(x, n)
    z = x[:, 2]
    return 2.0 * omega * z - K * (n + 1) * (n + 2) * z * re


def rossby_haurwitz_paper(x, k=4, w=None, Omega=OMEGA_EARTH_DAY):
    """The paper's form (Sec. 4, Rossby-Haurwitz wave):
    zeta = 2 w sin(theta) + (k^2+3k+2) sin(theta) cos^k(theta) cos(k phi), with
    theta the latitude.  w defaults to the stationary choice 2 Omega/(k(k+3))
    (zero phase speed), which for k = 4 gives 2w = 2 pi / 7 per day."""
    if w is None:
        w = 2.0 * Omega / (k * (k + 3))
    re, _ = _re_im_pow(x, k)
    z = x[:, 2]
    return 2.0 * w * z + (k * k + 3 * k + 2) * z * re


def great_circle_distance(x, c):
    cr = np.cross(x, c[None, :])
    return np.arctan2(np.sqrt((cr * cr).sum(1)), x @ c)


def gaussian_vortex(x, seed, width=0.1, amplitude=1.0, noise=1e-3):
    """Gaussian vortex zeta = a exp(-(d/width)^2) + U(-noise, noise), with d the
    great-circle distance to a seeded random centre (normalised standard
    normal 3-vector).  Not mean-corrected."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(3)
    c = c / np.sqrt((c * c).sum())
    d = great_circle_distance(x, c)
    z = amplitude * np.exp(-(d / width) ** 2)
    if noise:
        z = z + rng.uniform(-noise, noise, size=len(x))
    return z


def gaussian_vortex_paper(x, areas, lon_c=0.0, lat_c=np.pi / 20):
    """The paper's Gaussian vortex (Sec. 4): 4 pi exp(-16 |x - x_c|^2) + C per
    day, C chosen so that sum(zeta A) = 0."""
    c = np.array([np.cos(lat_c) * np.cos(lon_c), np.cos(lat_c) * np.sin(lon_c),
                  np.sin(lat_c)])
    d2 = ((x - c[None, :]) ** 2).sum(1)
    z = 4.0 * np.pi * np.exp(-16.0 * d2)
    return z - (z * areas).sum() / areas.sum()


def gaussian_pair(x, seed, width=0.1, amplitude=4.0 * np.pi / 86400.0):
    """A +/- pair of Gaussian vortices at two seeded random centres."""
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((2, 3))
    c = c / np.sqrt((c * c).sum(1))[:, None]
    d1 = great_circle_distance(x, c[0])
    d2 = great_circle_distance(x, c[1])
    return amplitude * (np.exp(-(d1 / width) ** 2) - np.exp(-(d2 / width) ** 2))


def polar_vortex(x, beta=1.5, lat0=15.0 * np.pi / 32.0):
    """Initial vorticity of the polar-vortex collapse experiment (Sec. 4.4), a
    zonally symmetric profile of latitude theta (per day, Omega = 2 pi per day):
    pi exp(-2 beta^2 (1 - cos(theta0 - theta))) (2 beta^2 cos(theta) sin(theta0 - theta) + sin(theta))."""
    lat = np.arcsin(np.clip(x[:, 2], -1.0, 1.0))
    b2 = 2.0 * beta * beta
    return np.pi * np.exp(-b2 * (1.0 - np.cos(lat0 - lat))) * (b2 * np.cos(lat) * np.sin(lat0 - lat) + np.sin(lat))
