"""GPU RK4 (Sec. 2 discrete system, Sec. 4 time stepping): graph-captured
steps against the eager path, and the Rossby-Haurwitz wave at N = 163842
against its closed-form propagation."""

import sys

import numpy as np
import pytest

import synthetic as S
from oracle import metrics

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_graph_steps_match_eager_bitwise(stc_lib):
    x0 = S.icosahedral_grid(5) @ S.random_rotation(8).T
    z0 = S.rossby_haurwitz(x0, 4)
    a = S.uniform_areas(len(x0))
    n = len(x0)
    kw = dict(theta=0.7, degree=8, n_crit=64, precision="fp32", denominator="dist2")
    cg = stc_lib.Context(n, **kw)
    ce = stc_lib.Context(n, eager_rk4=True, **kw)
    xg, zg = torch.from_numpy(x0.copy()).cuda(), torch.from_numpy(z0.copy()).cuda()
    xe, ze = torch.from_numpy(x0.copy()).cuda(), torch.from_numpy(z0.copy()).cuda()
    ad = torch.from_numpy(a).cuda()
    probe = torch.from_numpy(x0).cuda()
    for step in range(4):
        say(f"rk4 graph replay {step}")
        cg.rk4(xg, zg, ad, 1800.0, S.OMEGA_EARTH_S, 1)
        cg.sync()
        ce.rk4(xe, ze, ad, 1800.0, S.OMEGA_EARTH_S, 1)
        ce.sync()
        assert torch.equal(xg, xe) and torch.equal(zg, ze), step
        # eager work of the program between replays
        cg.velocity(probe, ze, ad)
        cg.sync()
    cg.close()
    ce.close()


def _phase(x, z, a, n):
    return np.angle(((x[:, 0] + 1j * x[:, 1]) ** n * x[:, 2] * z * a).sum())


def _run(stc_lib, x0, z0, a, dt, Om, steps, precision="fp64", theta=0.7, degree=8):
    ctx = stc_lib.Context(len(x0), theta=theta, degree=degree, n_crit=64, precision=precision,
                          denominator="dist2")
    xd, zd, ad = (torch.from_numpy(v.copy()).cuda() for v in (x0, z0, a))
    for block in range(0, steps, 48):
        ctx.rk4(xd, zd, ad, dt, Om, min(48, steps - block))
        ctx.sync()
        say(f"  step {min(block + 48, steps)} of {steps}")
    x, z = xd.cpu().numpy(), zd.cpu().numpy()
    ctx.close()
    return x, z


# Particles are advected without remeshing, so the quadrature error grows as
# the point set distorts (E_N ~ 3e-3 after one day at N = 163842, ~0.25 after
# ten); the closed-form checks below therefore run for one day, where the
# distortion is small and the error still falls with N.
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_rossby_haurwitz_one_day(stc_lib, precision):
    wl = S.make_workload("rh4_l7")
    x0, z0, a = wl["x"], wl["zeta"], wl["area"]
    omega = K = 7.848e-6
    Om = S.OMEGA_EARTH_S
    dt, steps = wl["dt"], 48
    say(f"RH n=4 N={len(x0)} {steps} steps {precision}")
    x, z = _run(stc_lib, x0, z0, a, dt, Om, steps, precision)
    T = dt * steps
    nu = (4 * (3 + 4) * omega - 2 * Om) / ((1 + 4) * (2 + 4))   # Sec. 4 phase speed, k = 4
    expected = nu * T          # 12.26 degrees: no 90-degree alias of the k = 4 pattern
    shift = np.angle(np.exp(1j * (_phase(x, z, a, 4) - _phase(x0, z0, a, 4)))) / 4
    say(f"  shift {np.degrees(shift):.4f} deg, closed form {np.degrees(expected):.4f} deg")
    assert abs(shift - expected) < 2e-3 * abs(expected)
    # vorticity against the exact solution rotated by nu T
    c, s_ = np.cos(-expected), np.sin(-expected)
    R = np.array([[c, -s_, 0], [s_, c, 0], [0, 0, 1]])
    z_exact = S.rossby_haurwitz(x @ R.T, 4, omega=omega, K=K)
    en = metrics.rel_l2_scalar(z, z_exact, a)
    drift = abs((z * a).sum() - (z0 * a).sum()) / (np.abs(z0) * a).sum()
    say(f"  E_N {en:.3e} circulation drift {drift:.2e}")
    assert np.isfinite(x).all() and np.isfinite(z).all()
    assert en < 6e-3
    assert drift < 1e-3
    # particles stay on the sphere (renormalised each step)
    assert np.abs(np.linalg.norm(x, axis=1) - 1).max() < 1e-14


def test_stationary_rossby_haurwitz_converges(stc_lib):
    """The paper's stationary k = 4 wave (zero phase speed, time in days):
    the vorticity carried by the particles should stay zeta_0(x_i); the
    one-day error E_N falls by more than 2x per grid level."""
    errs = []
    for L in (5, 6, 7):
        x0, faces = S.icosahedral_grid(L, return_faces=True)
        a = S.node_patch_areas(x0, faces)
        z0 = S.rossby_haurwitz_paper(x0)
        say(f"stationary RH L{L} N={len(x0)}")
        x, z = _run(stc_lib, x0, z0, a, 1.0 / 48, S.OMEGA_EARTH_DAY, 48)
        errs.append(metrics.rel_l2_scalar(z, S.rossby_haurwitz_paper(x), a))
        say(f"  E_N {errs[-1]:.3e}")
    assert errs[0] > 2 * errs[1] > 4 * errs[2]
    assert errs[2] < 1.5e-2


def test_rk4_rejects_the_dot_denominator(stc_lib):
    x = S.icosahedral_grid(2)
    ctx = stc_lib.Context(len(x), theta=0.7, degree=4, n_crit=8, denominator="dot")
    xd = torch.from_numpy(x.copy()).cuda()
    one = torch.ones(len(x), dtype=torch.float64, device="cuda")
    with pytest.raises(stc_lib.StcError):
        ctx.rk4(xd, one.clone(), one, 1.0, 0.0, 1)
    ctx.close()


def test_rossby_haurwitz_ten_days(stc_lib):
    """The configured run: RH n = 4 at N = 163842, dt = 1800 s, 480 steps.
    Particles are never remeshed, so the wave's phase lags the closed form by
    a discretisation error of the particle set: -2.3% at level 7 and -4.8% at
    level 6 (halving per level), while a much tighter tree (theta 0.4, d 12)
    moves the phase by 0.15 degrees only -- the tree's approximation does not
    set the lag.  Bars: lag within 3% at level 7 and at least 1.5x larger at
    level 6; tree control within 0.5 degrees; FP32 within 0.1 degrees of
    FP64; relative circulation drift below 1e-3."""
    import bench
    wl = S.make_workload("rh4_l7")
    x0, z0, a = wl["x"], wl["zeta"], wl["area"]
    dt, steps, Om = wl["dt"], wl["steps"], S.OMEGA_EARTH_S
    omega = 7.848e-6
    nu = (4 * 7 * omega - 2 * Om) / 30.0
    expected = np.degrees(nu * dt * steps)
    res = {}
    for tag, prec, th, d in (("fp64", "fp64", 0.7, 8), ("fp32", "fp32", 0.7, 8), ("ctrl", "fp64", 0.4, 12)):
        say(f"RH ten days {tag}")
        x, z, ph, _ = bench.rh_ten_day_run(stc_lib, x0, z0, a, dt, Om, steps, prec, th, d, log=say)
        drift = abs((z * a).sum() - (z0 * a).sum()) / (np.abs(z0) * a).sum()
        res[tag] = (np.degrees(ph[-1] - ph[0]) / 4, drift)
        say(f"  phase {res[tag][0]:.3f} deg (closed form {expected:.3f}), drift {drift:.2e}")
        assert np.isfinite(x).all() and np.isfinite(z).all()
    x6, f6 = S.icosahedral_grid(6, return_faces=True)
    a6 = S.node_patch_areas(x6, f6)
    z6 = S.rossby_haurwitz(x6, 4)
    say("RH ten days level 6")
    _, _, ph6, _ = bench.rh_ten_day_run(stc_lib, x6, z6, a6, dt, Om, steps, "fp64", 0.7, 8, log=say)
    lag6 = expected - np.degrees(ph6[-1] - ph6[0]) / 4
    lag7 = expected - res["fp64"][0]
    say(f"  lag level 6 {lag6:.3f} deg, level 7 {lag7:.3f} deg")
    assert 0 < lag7 < 0.03 * expected
    assert lag6 > 1.5 * lag7
    assert abs(res["ctrl"][0] - res["fp64"][0]) < 0.5
    assert abs(res["fp32"][0] - res["fp64"][0]) < 0.1
    assert res["fp64"][1] < 1e-3 and res["fp32"][1] < 1e-3
