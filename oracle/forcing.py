"""O4: vorticity forcing of the polar-vortex collapse experiment (Sec. 4.4,
polar vortex collapse).  TEST INFRASTRUCTURE ONLY.

The forced Biot-Savart integral replaces zeta by zeta - F_R in the source
charges, so the discrete system uses q_j = (zeta_j - F_R(x_j, t)) A_j; the
particles' own zeta still evolves by dzeta/dt = -2 Omega u_z.

    A(t)   ramp: (1 - cos(pi t / T_p)) / 2 on [0, T_p), 1 on [T_p, T_f - T_p),
           (1 - cos(pi + pi (t - T_f + T_p) / T_p)) / 2 on [T_f - T_p, T_f),
           0 from T_f on (and, reading, 0 before t = 0);
    B(lat) tan^2(lat1) / tan^2(lat) * exp(1 - tan^2(lat1) / tan^2(lat)) for
           0 < lat <= pi/2, else 0;
    F_R    (3/5) Omega k^2 A(t) B(lat) cos(k lon).

Latitude and longitude of a particle come from the direction of x (stage
points of RK4 lie slightly off the sphere): lat = arcsin(z / |x|),
lon = arctan2(y, x).  Written with the library's trigonometric functions,
exactly in the paper's notation.
"""

import numpy as np


def ramp(t, t_ramp, t_total):
    """A(t) of the forcing (Sec. 4.4, polar vortex collapse), for scalar t."""
    t = float(t)
    if t < 0.0:
        return 0.0
    if t < t_ramp:
        return (1.0 - np.cos(t / t_ramp * np.pi)) / 2.0
    if t < t_total - t_ramp:
        return 1.0
    if t < t_total:
        return (1.0 - np.cos(np.pi + (t - t_total + t_ramp) / t_ramp * np.pi)) / 2.0
    return 0.0


def latitude_profile(lat, lat1):
    """B(lat): zero on the southern hemisphere and the equator."""
    lat = np.asarray(lat, dtype=np.float64)
    out = np.zeros_like(lat)
    north = lat > 0.0
    ratio = np.tan(lat1) ** 2 / np.tan(lat[north]) ** 2
    out[north] = ratio * np.exp(1.0 - ratio)
    return out


def lat_lon(x):
    x = np.asarray(x, dtype=np.float64)
    r = np.sqrt((x * x).sum(1))
    return np.arcsin(np.clip(x[:, 2] / r, -1.0, 1.0)), np.arctan2(x[:, 1], x[:, 0])


def forcing(x, t, k, omega, lat1, t_ramp, t_total):
    """F_R(x_j, t) at every particle."""
    lat, lon = lat_lon(x)
    amp = 3.0 / 5.0 * omega * k * k * ramp(t, t_ramp, t_total)
    return amp * latitude_profile(lat, lat1) * np.cos(k * lon)


def forced_zeta(x, zeta, t, k, omega, lat1, t_ramp, t_total):
    """zeta - F_R: the field whose charges the forced velocity uses."""
    return np.asarray(zeta, dtype=np.float64) - forcing(x, t, k, omega, lat1, t_ramp, t_total)


def rk4_step(x, zeta, area, t, dt, omega, velocity_fn, forcing_args, project=True):
    """One classical RK4 step of the forced system; stage s sees F_R at time
    t + c_s dt with c = (0, 1/2, 1/2, 1).  forcing_args = (k, lat1, T_p, T_f);
    the forcing's Omega is the rotation rate `omega`."""
    k, lat1, t_ramp, t_total = forcing_args

    def rhs(xs, zs, ts):
        u = velocity_fn(xs, forced_zeta(xs, zs, ts, k, omega, lat1, t_ramp, t_total), area)
        return u, -2.0 * omega * u[:, 2]

    k1x, k1z = rhs(x, zeta, t)
    k2x, k2z = rhs(x + 0.5 * dt * k1x, zeta + 0.5 * dt * k1z, t + 0.5 * dt)
    k3x, k3z = rhs(x + 0.5 * dt * k2x, zeta + 0.5 * dt * k2z, t + 0.5 * dt)
    k4x, k4z = rhs(x + dt * k3x, zeta + dt * k3z, t + dt)
    xn = x + (dt / 6.0) * (k1x + 2.0 * k2x + 2.0 * k3x + k4x)
    zn = zeta + (dt / 6.0) * (k1z + 2.0 * k2z + 2.0 * k3z + k4z)
    if project:
        xn = xn / np.sqrt((xn * xn).sum(1))[:, None]
    return xn, zn
