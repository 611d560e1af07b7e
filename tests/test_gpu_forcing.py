"""GPU vorticity forcing (Sec. 4.4, polar vortex collapse) against the oracle:
the forced velocity of one evaluation, the forcing switched off by its ramp,
and forced RK4 steps (eager and graph-captured) across the end of the ramp-up,
with the forcing clock advanced by the steps."""

import sys

import numpy as np
import pytest

import synthetic as S
from oracle import forcing as oforce
from oracle import tree as otree

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

OM = S.OMEGA_EARTH_DAY
LAT1, TP, TF = np.pi / 3.0, 4.0, 15.0


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("k,t", [(1, 2.5), (2, 9.0), (2, 13.2)])
def test_forced_velocity_matches_oracle(stc_lib, k, t):
    x = S.icosahedral_grid(4) @ S.random_rotation(21).T
    z = S.polar_vortex(x)
    a = S.uniform_areas(len(x))
    th, d, nc = 0.7, 6, 32
    ctx = stc_lib.Context(len(x), theta=th, degree=d, n_crit=nc, max_level=4)
    ctx.set_forcing(k, OM, LAT1, TP, TF, time=t)
    say(f"forced velocity k={k} t={t} N={len(x)}")
    u = ctx.velocity(dev(x), dev(z), dev(a)).cpu().numpy()
    ctx.sync()
    zf = oforce.forced_zeta(x, z, t, k, OM, LAT1, TP, TF)
    ref = otree.velocity(x, zf, a, theta=th, degree=d, n_crit=nc, max_level=4)
    plain = otree.velocity(x, z, a, theta=th, degree=d, n_crit=nc, max_level=4)
    scale = np.abs(ref).max()
    assert np.abs(u - ref).max() / scale < 1e-10
    assert np.abs(plain - ref).max() / scale > 1e-3  # the forcing changes the result
    on, f = ctx.forcing()
    assert on and f["k"] == k and f["time"] == t
    ctx.close()


def test_forcing_outside_its_window_changes_nothing(stc_lib):
    x = S.icosahedral_grid(4)
    z = S.polar_vortex(x)
    a = S.uniform_areas(len(x))
    ctx = stc_lib.Context(len(x), theta=0.7, degree=6, n_crit=32, precision="fp32", denominator="dist2")
    say("forcing off vs outside its window")
    u0 = ctx.velocity(dev(x), dev(z), dev(a)).clone()
    for t in (-1.0, TF, TF + 2.0):
        ctx.set_forcing(2, OM, LAT1, TP, TF, time=t)
        u1 = ctx.velocity(dev(x), dev(z), dev(a))
        assert torch.equal(u0, u1), t
    ctx.clear_forcing()
    assert not ctx.forcing()[0]
    ctx.close()


def test_invalid_forcing_is_rejected(stc_lib):
    ctx = stc_lib.Context(1000, theta=0.7, degree=6, n_crit=32)
    for args in [(17, OM, LAT1, TP, TF), (-1, OM, LAT1, TP, TF), (1, OM, 0.0, TP, TF), (1, OM, 1.6, TP, TF),
                 (1, OM, LAT1, 0.0, TF), (1, OM, LAT1, TP, 7.9), (1, float("nan"), LAT1, TP, TF)]:
        with pytest.raises(stc_lib.StcError):
            ctx.set_forcing(*args)
    assert not ctx.forcing()[0]
    ctx.close()


@pytest.mark.parametrize("eager", [True, False])
def test_forced_rk4_matches_oracle(stc_lib, eager):
    """Three steps of dt = 0.05 days from t = 3.92: the stages straddle the end
    of the ramp-up at T_p = 4 (an error in a stage time changes A there)."""
    x0 = S.icosahedral_grid(4) @ S.random_rotation(22).T
    z0 = S.polar_vortex(x0)
    a = S.uniform_areas(len(x0))
    th, d, nc, k = 0.7, 6, 32, 2
    t0, dt, steps = 3.92, 0.05, 3
    vel = lambda xx, zz, aa: otree.velocity(xx, zz, aa, theta=th, degree=d, n_crit=nc, max_level=4, den="dist2")
    xr, zr, t = x0, z0, t0
    for _ in range(steps):
        xr, zr = oforce.rk4_step(xr, zr, a, t, dt, OM, vel, (k, LAT1, TP, TF))
        t += dt
    say(f"forced rk4 eager={eager} N={len(x0)} {steps} steps")
    ctx = stc_lib.Context(len(x0), theta=th, degree=d, n_crit=nc, max_level=4, denominator="dist2",
                          eager_rk4=eager)
    ctx.set_forcing(k, OM, LAT1, TP, TF, time=t0)
    xg, zg = dev(x0.copy()), dev(z0.copy())
    ctx.rk4(xg, zg, dev(a), dt, OM, 1)       # one call of one step, then one of two:
    ctx.rk4(xg, zg, dev(a), dt, OM, steps - 1)  # the clock carries over (and the graph is replayed)
    ctx.sync()
    assert ctx.forcing()[1]["time"] == pytest.approx(t0 + steps * dt, abs=1e-12)
    xg, zg = xg.cpu().numpy(), zg.cpu().numpy()
    assert np.abs(xg - xr).max() < 1e-11
    assert np.abs(zg - zr).max() < 1e-10 * np.abs(z0).max()
    ctx.close()


@pytest.mark.parametrize("k", [0, 1, 2, 5])
def test_forcing_field_matches_oracle(stc_lib, k):
    """stc_forcing_field against the oracle's trigonometric form, on the
    sphere and off it (scaled rows), at the ramp's pieces; poles, the equator
    and the southern hemisphere included."""
    x = np.concatenate([S.random_sphere_points(5000, 31), [[0, 0, 1.0], [0, 0, -1.0], [1.0, 0, 0], [0, 1.0, 0]]])
    x = x * np.linspace(0.9, 1.1, len(x))[:, None]
    xd = dev(x)
    for t in (-0.5, 1.3, 4.0, 8.0, 12.7, 15.0):
        say(f"forcing field k={k} t={t}")
        got = stc_lib.forcing_field(xd, k, OM, LAT1, TP, TF, t).cpu().numpy()
        want = oforce.forcing(x, t, k, OM, LAT1, TP, TF)
        scale = 0.6 * OM * max(k, 1) ** 2
        assert np.abs(got - want).max() <= 1e-13 * scale, t
        assert got[-4] == 0.0 and got[-3] == 0.0 and got[-2] == 0.0


def test_forced_rk4_batched_bitwise_equal_single(stc_lib):
    """The forcing acts on every member of an ensemble: forced batched steps
    equal forced steps of each member alone, bitwise, and the clock advances
    once per step."""
    ens = S.make_ensemble(members=3, seed0=4, levels=(4, 5))
    off = ens["offsets"]
    kw = dict(theta=0.7, degree=6, n_crit=32, precision="fp32", denominator="dist2")
    t0, dt, steps = 3.95, 0.02, 3
    say(f"forced rk4 batch N={off[-1]}")
    cb = stc_lib.Context(int(off[-1]), members=len(off) - 1, n_max_member=int(np.diff(off).max()), **kw)
    cb.set_forcing(1, OM, LAT1, TP, TF, time=t0)
    xb, zb, ab = dev(ens["x"]), dev(ens["zeta"]), dev(ens["area"])
    cb.rk4_batched(xb, zb, ab, off, dt, OM, steps)
    cb.sync()
    assert cb.forcing()[1]["time"] == pytest.approx(t0 + steps * dt, abs=1e-12)
    for m in range(len(off) - 1):
        sl = slice(off[m], off[m + 1])
        cs = stc_lib.Context(int(off[m + 1] - off[m]), max_level=cb.max_level, **kw)
        cs.set_forcing(1, OM, LAT1, TP, TF, time=t0)
        xs, zs = dev(ens["x"][sl]), dev(ens["zeta"][sl])
        cs.rk4(xs, zs, dev(ens["area"][sl]), dt, OM, steps)
        cs.sync()
        assert torch.equal(xb[sl], xs) and torch.equal(zb[sl], zs), m
        cs.close()
    cb.close()
