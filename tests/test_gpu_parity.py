"""GPU parity: the HIP library through its C ABI against the CPU oracle on the
same seeded inputs.

Bars: tree permutation, node counts and the four interaction lists
bit-exact; FP64 velocities within 1e-10 relative (max norm over the largest
velocity) of the oracle running the same algorithm; FP32 within the bound
derived for the precision form.
"""

import functools
import sys

import numpy as np
import pytest

import synthetic as S
from oracle import direct as odirect
from oracle import metrics
from oracle import tree as otree
from oracle import rk4 as ork4

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# ---- cases -------------------------------------------------------------------------

def _case(name):
    if name == "grid_l5":           # every particle on tree edges (exact ties)
        x = S.icosahedral_grid(5)
        z = S.rossby_haurwitz(x, 4)
    elif name in ("rotated_l4", "rotated_l4_d12"):
        x = S.icosahedral_grid(4) @ S.random_rotation(11).T
        z = S.rossby_haurwitz(x, 3)
    elif name == "random_7001":     # ragged leaves
        x = S.random_sphere_points(7001, 5)
        z = S.gaussian_vortex(x, seed=5)
    elif name == "clustered_6000":  # depth limit reached, leaves above N_T
        x = S.clustered_sphere_points(6000, 9, width=0.004)
        z = S.gaussian_vortex(x, seed=9)
    elif name == "planes_3000":     # a coordinate exactly 0: on the root edges that lie in
        x = S.random_sphere_points(3000, 7)   # coordinate planes (orientation exactly 0)
        x[np.arange(3000) % 3 == 0, 0] = 0.0
        x[np.arange(3000) % 3 == 1, 1] = 0.0
        x /= np.linalg.norm(x, axis=1)[:, None]
        z = S.gaussian_vortex(x, seed=7)
    elif name == "tiny_50":
        x = S.random_sphere_points(50, 1)
        z = np.random.default_rng(1).standard_normal(50)
    else:
        raise KeyError(name)
    return x, z, S.uniform_areas(len(x))


CASES = {
    # name: (theta, degree, n_crit, max_level)
    "grid_l5": (0.7, 8, 64, None),
    "rotated_l4": (0.7, 6, 32, None),
    "random_7001": (0.6, 5, 20, None),
    "clustered_6000": (0.8, 4, 24, 4),
    "tiny_50": (0.7, 3, 4, None),
    "planes_3000": (0.7, 5, 16, None),
    "rotated_l4_d12": (0.7, 12, 96, None),  # 91 proxy points: the coefficient kernel for more than 66
}

# Denominator for the FP64 parity of each case.  The literal 1 - x.y loses
# about log10(2 / (1 - x.y)) digits for close pairs: on the random and
# clustered sets (closest pairs 5e-5 and 4e-6 apart) the oracle's own two
# denominators already differ by 4e-9 and 2e-7, so those cases compare in the
# |x - y|^2 / 2 form (the paper's remedy, Sec. 2), whose rounding error
# does not grow as pairs approach.
CASE_DEN = {"grid_l5": "dot", "rotated_l4": "dot", "random_7001": "dist2", "clustered_6000": "dist2",
            "tiny_50": "dot", "planes_3000": "dist2", "rotated_l4_d12": "dot"}


@functools.lru_cache(maxsize=None)
def oracle_tree(name, den="dot"):
    x, z, a = _case(name)
    th, d, nc, ml = CASES[name]
    return otree.TreeCode(x, z, a, theta=th, degree=d, n_crit=nc, max_level=ml, den=den)


def gpu_ctx(stc, name, precision="fp64", den="dot"):
    x, z, a = _case(name)
    th, d, nc, ml = CASES[name]
    ctx = stc.Context(len(x), theta=th, degree=d, n_crit=nc, max_level=-1 if ml is None else ml,
                      precision=precision, denominator=den)
    return ctx, x, z, a


# ---- direct sum ---------------------------------------------------------------------

@pytest.mark.parametrize("den", ["dot", "dist2"])
def test_direct_fp64_full(stc_lib, den):
    x = S.icosahedral_grid(5)
    z = S.rossby_haurwitz(x, 4)
    a = S.uniform_areas(len(x))
    say(f"direct fp64 {den} N={len(x)}")
    u = stc_lib.direct(dev(x), dev(z), dev(a), denominator=den).cpu().numpy()
    ref = odirect.velocity(x, z, a, den=den)
    assert np.abs(u - ref).max() / np.abs(ref).max() < 1e-12


@pytest.mark.parametrize("den,tol", [("dist2", 1e-12), ("dot", 2e-11)])
def test_direct_subset_ragged(stc_lib, den, tol):
    """Random points: with 1 - x.y the oracle's two denominators already
    differ by 3.5e-12 here (cancellation for close pairs), hence the looser
    bar for that form."""
    x = S.random_sphere_points(40961, 3)
    z = S.gaussian_vortex(x, seed=3)
    a = S.uniform_areas(len(x))
    idx = S.subset_indices(len(x), 333, 4)
    say(f"direct subset N=40961 m=333 {den}")
    u = stc_lib.direct(dev(x), dev(z), dev(a), targets=dev(idx), denominator=den).cpu().numpy()
    ref = odirect.velocity(x, z, a, targets=idx, den=den)
    assert np.abs(u - ref).max() / np.abs(ref).max() < tol


def test_direct_fp32_error_bound(stc_lib):
    x = S.icosahedral_grid(5)
    z = S.gaussian_vortex(x, seed=2)
    a = S.uniform_areas(len(x))
    say("direct fp32 N=10242")
    u = stc_lib.direct(dev(x), dev(z), dev(a), precision="fp32", denominator="dist2").cpu().numpy()
    ref = odirect.velocity(x, z, a)
    assert metrics.rel_l2_velocity(u, ref, a) < 2e-6


# ---- tree build and lists -------------------------------------------------------------

@pytest.mark.parametrize("name", list(CASES))
def test_tree_and_lists_bit_exact(stc_lib, name):
    ot = oracle_tree(name)
    ctx, x, z, a = gpu_ctx(stc_lib, name)
    say(f"tree+lists {name} N={len(x)} L={ctx.max_level}")
    assert ctx.max_level == ot.max_level
    ctx.tree_build(dev(x))
    ctx.upward(dev(z), dev(a))
    ctx.traverse()
    perm, cnt = ctx.copy_tree()
    np.testing.assert_array_equal(perm, ot.ptree.perm)
    np.testing.assert_array_equal(cnt, ot.ptree.count)
    for kind in ("PP", "PC", "CP", "CC"):
        got = ctx.copy_list(kind)
        np.testing.assert_array_equal(got, ot.lists[kind].reshape(-1, 2), err_msg=kind)
    counts, evals = ctx.list_counts()
    assert counts == ot.list_counts()
    assert sum(evals.values()) == ot.kernel_evaluations()
    ctx.close()


@pytest.mark.parametrize("name", ["grid_l5", "random_7001", "clustered_6000"])
def test_proxy_charges(stc_lib, name):
    ot = oracle_tree(name)
    ctx, x, z, a = gpu_ctx(stc_lib, name)
    say(f"proxy charges {name}")
    ctx.tree_build(dev(x))
    ctx.upward(dev(z), dev(a))
    big = np.nonzero(ot.ptree.count > ot.n_crit)[0]
    rng = np.random.default_rng(0)
    for node in rng.choice(big, size=min(12, len(big)), replace=False):
        w = ctx.proxy_charges(int(node))
        ref = ot.proxy_charges(int(node))
        assert np.abs(w - ref).max() <= 1e-10 * np.abs(ref).max(), node
    ctx.close()


def test_proxy_charges_multi_item(stc_lib):
    """Nodes with more particles than one upward-pass item holds (2048): each
    item writes its partial sums, and a separate finishing kernel adds a
    node's items in a fixed order.  A second upward pass with doubled
    vorticity must give exactly doubled charges (no state carries over from
    the first pass)."""
    n = 60000
    x = S.random_sphere_points(n, 8)
    z = S.gaussian_vortex(x, seed=8)
    a = S.uniform_areas(n)
    ot = otree.TreeCode(x, z, a, theta=0.9, degree=5, n_crit=32, max_level=4)
    ctx = stc_lib.Context(n, theta=0.9, degree=5, n_crit=32, max_level=4)
    say("proxy charges, multi-item nodes N=60000")
    ctx.tree_build(dev(x))
    ctx.upward(dev(z), dev(a))
    multi = np.nonzero(ot.ptree.count > 2048)[0]
    assert len(multi) >= 10
    big = np.nonzero(ot.ptree.count > ot.n_crit)[0]
    nodes = list(multi) + list(np.random.default_rng(1).choice(big, 10, replace=False))
    first = {}
    for node in nodes:
        w = ctx.proxy_charges(int(node))
        ref = ot.proxy_charges(int(node))
        assert np.abs(w - ref).max() <= 1e-10 * np.abs(ref).max(), node
        first[int(node)] = w
    ctx.upward(dev(2.0 * z), dev(a))
    for node in nodes:
        np.testing.assert_array_equal(ctx.proxy_charges(int(node)), 2.0 * first[int(node)])
    ctx.close()


# ---- velocities -------------------------------------------------------------------------

@pytest.mark.parametrize("name", list(CASES))
def test_velocity_fp64_matches_oracle_tree(stc_lib, name):
    den = CASE_DEN[name]
    ot = oracle_tree(name, den=den)
    ctx, x, z, a = gpu_ctx(stc_lib, name, den=den)
    say(f"velocity fp64 {name} {den}")
    u = ctx.velocity(dev(x), dev(z), dev(a)).cpu().numpy()
    ref = ot.velocity()
    scale = np.abs(ref).max()
    assert np.abs(u - ref).max() / scale < 1e-10
    # near and far separately
    un = ctx.eval_near().cpu().numpy()
    uf = ctx.eval_far().cpu().numpy()
    rn = ot.velocity(parts=("near",))
    rf = ot.velocity(parts=("far",))
    assert np.abs(un - rn).max() / scale < 1e-10
    assert np.abs(uf - rf).max() / scale < 1e-10
    # accumulate flag: near + far = full
    ua = ctx.eval_near()
    ctx.eval_far(out=ua, accumulate=True)
    assert np.abs(ua.cpu().numpy() - ref).max() / scale < 1e-10
    ctx.close()


def test_velocity_fp64_dist2(stc_lib):
    name = "grid_l5"
    ot = oracle_tree(name, den="dist2")
    ctx, x, z, a = gpu_ctx(stc_lib, name, den="dist2")
    say("velocity fp64 dist2")
    u = ctx.velocity(dev(x), dev(z), dev(a)).cpu().numpy()
    ref = ot.velocity()
    assert np.abs(u - ref).max() / np.abs(ref).max() < 1e-10
    ctx.close()


@pytest.mark.parametrize("name", ["grid_l5", "random_7001", "rotated_l4_d12"])
def test_velocity_fp32_precision_form(stc_lib, name):
    """FP32 sums with target-relative coordinates: the difference from the
    FP64 tree is rounding only (the lists are identical)."""
    ot = oracle_tree(name, den="dist2")
    ctx, x, z, a = gpu_ctx(stc_lib, name, precision="fp32", den="dist2")
    say(f"velocity fp32 {name}")
    u = ctx.velocity(dev(x), dev(z), dev(a)).cpu().numpy()
    ref = ot.velocity()
    assert metrics.rel_l2_velocity(u, ref, a) < 1e-6
    ctx.close()


def test_degenerate_sizes(stc_lib):
    ctx = stc_lib.Context(100, theta=0.7, degree=4, n_crit=8)
    # one particle: no pair, zero velocity
    x = S.random_sphere_points(1, 0)
    say("degenerate N=1")
    u = ctx.velocity(dev(x), dev(np.ones(1)), dev(np.ones(1))).cpu().numpy()
    np.testing.assert_array_equal(u, 0.0)
    # two particles: the direct sum
    x = S.random_sphere_points(2, 1)
    z = np.array([1.0, -2.0])
    a = np.array([0.5, 0.25])
    say("degenerate N=2")
    u = ctx.velocity(dev(x), dev(z), dev(a)).cpu().numpy()
    np.testing.assert_allclose(u, odirect.velocity(x, z, a), rtol=1e-13, atol=1e-16)
    # zero particles: a no-op
    say("degenerate N=0")
    out = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    ctx.velocity(torch.zeros((0, 3), dtype=torch.float64, device="cuda"),
                 torch.zeros(0, dtype=torch.float64, device="cuda"),
                 torch.zeros(0, dtype=torch.float64, device="cuda"), out=out)
    ctx.sync()
    # n above n_max is rejected on the host
    with pytest.raises(stc_lib.StcError):
        x = S.random_sphere_points(101, 1)
        ctx.velocity(dev(x), dev(np.ones(101)), dev(np.ones(101)))
    ctx.close()


def test_capacity_overflow_is_reported(stc_lib):
    x = S.random_sphere_points(3000, 2)
    ctx = stc_lib.Context(3000, theta=0.7, degree=4, n_crit=8, list_capacity=64)
    say("capacity overflow")
    ctx.velocity(dev(x), dev(np.ones(3000)), dev(np.ones(3000)))
    with pytest.raises(stc_lib.StcError) as e:
        ctx.sync()
    assert e.value.status == 2
    ctx.close()


def test_nonfinite_position_is_reported(stc_lib):
    x = S.random_sphere_points(2000, 4)
    x[777] = np.nan
    ctx = stc_lib.Context(2000, theta=0.7, degree=4, n_crit=16)
    say("non-finite position")
    ctx.velocity(dev(x), dev(np.ones(2000)), dev(np.ones(2000)))
    with pytest.raises(stc_lib.StcError) as e:
        ctx.sync()
    assert e.value.status == 7 and "non-finite particle position" in str(e.value)   # STC_ERR_NONFINITE
    # the same context then takes finite input again
    x[777] = S.random_sphere_points(1, 5)[0]
    u = ctx.velocity(dev(x), dev(np.ones(2000)), dev(np.ones(2000)))
    ctx.sync()
    assert np.isfinite(u.cpu().numpy()).all()
    # a non-finite vorticity or area is reported the same way (charge q = zeta A)
    for bad_z, bad_a in ((np.nan, 1.0), (1.0, np.inf)):
        z, a = np.ones(2000), np.ones(2000)
        z[123], a[123] = bad_z, bad_a
        say(f"non-finite charge zeta={bad_z} area={bad_a}")
        ctx.velocity(dev(x), dev(z), dev(a), out=u)
        with pytest.raises(stc_lib.StcError) as e:
            ctx.sync()
        assert e.value.status == 7 and "vorticity or area" in str(e.value)
    ctx.velocity(dev(x), dev(np.ones(2000)), dev(np.ones(2000)), out=u)
    ctx.sync()
    ctx.close()


def test_workspace_holds_every_device_buffer(stc_lib):
    """A context's device memory is the caller's workspace tensor (sized by
    stc_workspace_size): after a warm-up evaluation (the HIP runtime sets up
    its own structures on first launches), three further evaluations leave
    the device's free memory unchanged and repeat the first result bitwise."""
    x = S.random_sphere_points(20000, 11)
    z = S.random_sphere_points(20000, 12)[:, 0].copy()
    a = np.full(20000, 4 * np.pi / 20000)
    xd, zd, ad = dev(x), dev(z), dev(a)
    say("workspace: warm-up")
    ctx = stc_lib.Context(20000, theta=0.7, degree=6, n_crit=32, precision="fp32", denominator="dist2")
    assert ctx._ws.numel() == ctx.workspace_bytes
    u = ctx.velocity(xd, zd, ad)
    u2 = torch.empty_like(u)
    ctx.sync()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    say("workspace: measured evaluations")
    for _ in range(3):
        ctx.velocity(xd, zd, ad, out=u2)
    ctx.sync()
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, f"free device memory changed by {free0 - free1} bytes over three evaluations"
    assert torch.equal(u, u2)
    ctx.close()


def test_phase_timing_mask(stc_lib):
    ctx, x, z, a = gpu_ctx(stc_lib, "random_7001", precision="fp32", den="dist2")
    say("phase timing mask")
    u = ctx.velocity(dev(x), dev(z), dev(a))
    ctx.set_timing(3, phases=["near"])
    for _ in range(3):
        ctx.velocity(dev(x), dev(z), dev(a), out=u)
    ph, k = ctx.phase_times()
    assert k == 3 and ph["near"] > 0.0
    assert all(v == 0.0 for p, v in ph.items() if p != "near")
    ctx.set_timing(2)
    for _ in range(2):
        ctx.velocity(dev(x), dev(z), dev(a), out=u)
    ph, k = ctx.phase_times()
    assert k == 2 and all(v > 0.0 for v in ph.values())
    ctx.close()


def test_repeatable_bitwise(stc_lib):
    ctx, x, z, a = gpu_ctx(stc_lib, "random_7001", precision="fp32", den="dist2")
    say("repeatability")
    u1 = ctx.velocity(dev(x), dev(z), dev(a)).cpu().numpy()
    u2 = ctx.velocity(dev(x), dev(z), dev(a)).cpu().numpy()
    np.testing.assert_array_equal(u1, u2)
    ctx.close()


def test_rk4_matches_oracle(stc_lib):
    x0 = S.icosahedral_grid(4) @ S.random_rotation(2).T
    z0 = S.rossby_haurwitz(x0, 4)
    a = S.uniform_areas(len(x0))
    th, d, nc = 0.7, 6, 32
    Om = S.OMEGA_EARTH_S
    vel = lambda xx, zz, aa: otree.velocity(xx, zz, aa, theta=th, degree=d, n_crit=nc, max_level=4, den="dist2")
    say("rk4 2 steps N=2562")
    xr, zr = ork4.integrate(x0, z0, a, 1800.0, Om, 2, vel)
    ctx = stc_lib.Context(len(x0), theta=th, degree=d, n_crit=nc, max_level=4, denominator="dist2")
    xg, zg = dev(x0), dev(z0)
    ctx.rk4(xg, zg, dev(a), 1800.0, Om, 2)
    ctx.sync()
    xg, zg = xg.cpu().numpy(), zg.cpu().numpy()
    # The bar follows from the velocity bar (1e-10 of the largest velocity,
    # test_velocity_fp64_matches_oracle_tree): a step moves x by dt times a
    # weighted mean of four stage velocities (weights summing to one), so two
    # steps differ by at most 2 dt 1e-10 max|u|, plus feedback through the
    # stage positions that is smaller by dt |grad u| (about 0.1 here).
    # Likewise zeta moves by -2 Omega dt times a mean of stage u_z.
    umax = np.abs(vel(x0, z0, a)).max()
    bar_x = 1.1 * 2 * 1800.0 * 1e-10 * umax
    bar_z = 1.1 * 2 * 1800.0 * 2 * Om * 1e-10 * umax
    say(f"rk4: max |dx| {np.abs(xg - xr).max():.3e} (bar {bar_x:.3e}), max |dzeta| {np.abs(zg - zr).max():.3e} "
        f"(bar {bar_z:.3e})")
    assert np.abs(xg - xr).max() < bar_x
    assert np.abs(zg - zr).max() < bar_z
    ctx.close()


@pytest.mark.parametrize("precision,den", [("fp64", "dot"), ("fp32", "dist2")])
def test_velocity_graph_replays_equal_eager(stc_lib, precision, den):
    """stc_velocity_graph: every replay (with eager evaluations of the same
    context and synchronisations between replays, and the vorticity changed
    in place) is bitwise the eager evaluation of the same inputs; the
    replay's duration is positive."""
    x = S.random_sphere_points(7001, 21)
    a = np.full(7001, 4 * np.pi / 7001)
    kw = dict(theta=0.7, degree=6, n_crit=32, precision=precision, denominator=den)
    ctx = stc_lib.Context(7001, **kw)
    xd, ad = dev(x), dev(a)
    zd = dev(S.rossby_haurwitz(x, 4))
    ug = torch.empty((7001, 3), dtype=torch.float64, device="cuda")
    g = ctx.velocity_graph(xd, zd, ad, ug)
    for k in range(3):
        say(f"graph replay {k} {precision}")
        zd.copy_(dev(S.rossby_haurwitz(x, 3 + k) + 1e-3 * k))
        g.launch()
        torch.cuda.synchronize()
        assert g.last_ms() > 0
        ue = ctx.velocity(xd, zd, ad)          # eager work of the program between replays
        ctx.sync()
        assert torch.equal(ug, ue), k
    g.close()
    ctx.close()
