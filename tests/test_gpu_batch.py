"""GPU batching form: ensembles of independent particle sets evaluated in one
launch per phase (stc_create_batched / stc_velocity_batched /
stc_rk4_batched), through the C ABI.

Bars: every member's velocity, lists and RK4 state are bitwise those of a
single-member context with the same parameters (the member's work is the
same arithmetic in the same order); small members match the oracle tree to
1e-10 (FP64); the full 48-member ensemble matches the direct sum on sampled
targets within the tree code's error; launch shapes change results only at
rounding level.
"""

import sys

import numpy as np
import pytest

import synthetic as S
from oracle import tree as otree

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


KW = dict(theta=0.7, degree=6, n_crit=32)


def _small_ensemble(members=5, levels=(3, 4, 5)):
    return S.make_ensemble(members=members, seed0=4, levels=levels)


def _batched_ctx(stc_lib, ens, precision, den, **kw):
    off = ens["offsets"]
    n_member = int(np.diff(off).max())
    args = dict(KW)
    args.update(kw)
    return stc_lib.Context(int(off[-1]), members=len(off) - 1, n_max_member=n_member, precision=precision,
                           denominator=den, **args)


@pytest.mark.parametrize("precision,den", [("fp64", "dot"), ("fp64", "dist2"), ("fp32", "dist2")])
def test_members_bitwise_equal_single_contexts(stc_lib, precision, den):
    ens = _small_ensemble()
    off = ens["offsets"]
    say(f"batch {len(off) - 1} members N={off[-1]} {precision} {den}")
    cb = _batched_ctx(stc_lib, ens, precision, den)
    L = cb.max_level
    u = cb.velocity_batched(dev(ens["x"]), dev(ens["zeta"]), dev(ens["area"]), off).cpu().numpy()
    cb.sync()
    lists = {k: cb.copy_list(k) for k in stc_lib.LIST_NAMES}
    for m in range(len(off) - 1):
        sl = slice(off[m], off[m + 1])
        cs = stc_lib.Context(off[m + 1] - off[m], max_level=L, precision=precision, denominator=den, **KW)
        us = cs.velocity(dev(ens["x"][sl]), dev(ens["zeta"][sl]), dev(ens["area"][sl])).cpu().numpy()
        assert np.array_equal(u[sl], us), m
        for k in stc_lib.LIST_NAMES:
            mine = lists[k][cb.member_of_node(lists[k][:, 0]) == m]
            assert (cb.member_of_node(mine[:, 1]) == m).all()     # members never interact
            assert np.array_equal(cb.local_node(mine), cs.copy_list(k)), (m, k)
        cs.close()
    cb.close()


def test_small_members_match_oracle_tree(stc_lib):
    ens = _small_ensemble(members=3, levels=(3, 4))
    off = ens["offsets"]
    say(f"batch vs oracle N={off[-1]}")
    cb = _batched_ctx(stc_lib, ens, "fp64", "dot")
    u = cb.velocity_batched(dev(ens["x"]), dev(ens["zeta"]), dev(ens["area"]), off).cpu().numpy()
    for m in range(len(off) - 1):
        sl = slice(off[m], off[m + 1])
        ref = otree.TreeCode(ens["x"][sl], ens["zeta"][sl], ens["area"][sl], max_level=cb.max_level,
                             den="dot", **KW).velocity()
        assert np.abs(u[sl] - ref).max() / np.abs(ref).max() < 1e-10, m
    cb.close()


def test_tree_and_counts_per_member(stc_lib):
    ens = _small_ensemble(members=4, levels=(3, 4))
    off = ens["offsets"]
    cb = _batched_ctx(stc_lib, ens, "fp64", "dot")
    cb.tree_build_batched(dev(ens["x"]), off)
    perm, cnt = cb.copy_tree()
    for m in range(len(off) - 1):
        sl = slice(off[m], off[m + 1])
        pt = otree.TreeCode(ens["x"][sl], ens["zeta"][sl], ens["area"][sl], max_level=cb.max_level, **KW).ptree
        assert np.array_equal(perm[sl] - off[m], pt.perm)
        base = m << cb.node_bits
        assert np.array_equal(cnt[base:base + cb.nodes_per_member], pt.count)
    cb.close()


def test_rk4_batched_bitwise_equal_single(stc_lib):
    ens = _small_ensemble(members=4, levels=(4, 5))
    off = ens["offsets"]
    say(f"rk4 batch N={off[-1]}")
    cb = _batched_ctx(stc_lib, ens, "fp32", "dist2")
    xb, zb, ab = dev(ens["x"]), dev(ens["zeta"]), dev(ens["area"])
    cb.rk4_batched(xb, zb, ab, off, 1800.0, S.OMEGA_EARTH_S, 3)
    cb.sync()
    for m in range(len(off) - 1):
        sl = slice(off[m], off[m + 1])
        cs = stc_lib.Context(off[m + 1] - off[m], max_level=cb.max_level, precision="fp32", denominator="dist2", **KW)
        xs, zs = dev(ens["x"][sl]), dev(ens["zeta"][sl])
        cs.rk4(xs, zs, dev(ens["area"][sl]), 1800.0, S.OMEGA_EARTH_S, 3)
        cs.sync()
        assert torch.equal(xb[sl], xs) and torch.equal(zb[sl], zs), m
        cs.close()
    cb.close()


def test_launch_shapes_change_only_rounding(stc_lib):
    ens = _small_ensemble(members=4, levels=(4, 5))
    off = ens["offsets"]
    n = int(off[-1])
    for precision, tol in (("fp64", 1e-13), ("fp32", 1e-6)):
        cb = _batched_ctx(stc_lib, ens, precision, "dist2")
        x, z, a = dev(ens["x"]), dev(ens["zeta"]), dev(ens["area"])
        ref = cb.velocity_batched(x, z, a, off).cpu().numpy()
        scale = np.abs(ref).max()
        for shape in ((128, 8, 128, 8), (512, 4, 512, 16), (256, 24, 128, 4)):
            say(f"shape {shape} {precision}")
            cb.set_launch_config(n, *shape)
            assert cb.launch_config(n) == shape
            u = cb.velocity_batched(x, z, a, off).cpu().numpy()
            assert np.abs(u - ref).max() / scale < tol, shape
        # grid size alone moves no sum: bitwise
        cb.set_launch_config(n, 256, 5, 256, 7)
        assert np.array_equal(cb.velocity_batched(x, z, a, off).cpu().numpy(), ref)
        best = cb.autotune(repeats=2)
        say(f"autotuned {best}")
        assert cb.launch_config(n) == best
        u = cb.velocity_batched(x, z, a, off).cpu().numpy()
        assert np.abs(u - ref).max() / scale < tol
        cb.close()


def test_full_ensemble_against_direct_sum(stc_lib):
    """The configured ensemble: 48 members, N = 3.87e6 in total (levels
    5-7), FP32 precision form at the benchmark's setting (theta 0.8, d 10),
    24 graph-captured RK4 steps (dt = 1800 s) of all members together; then
    every member's velocity at its final state within the metric's 1e-6 of
    its FP64 direct sum on 256 seeded targets (the GPU direct sum, itself
    within 1e-12 of the oracle's), and 16 targets per member against the
    oracle's direct sum directly (bar 2e-6: fewer targets, more spread).  Three members also bitwise against single
    contexts before stepping."""
    import bench
    from oracle import direct as odirect
    ens = S.make_ensemble()
    off = ens["offsets"]
    M = len(off) - 1
    kw = dict(theta=bench.ENS_THETA, degree=bench.ENS_DEGREE, n_crit=bench.ENS_N_CRIT, precision="fp32",
              denominator="dist2")
    say(f"full ensemble M={M} N={off[-1]} {kw}")
    cb = stc_lib.Context(int(off[-1]), members=M, n_max_member=163842, **kw)
    x, z, a = dev(ens["x"]), dev(ens["zeta"]), dev(ens["area"])
    u = cb.velocity_batched(x, z, a, off)
    cb.sync()
    un = u.cpu().numpy()
    for m in (0, 7, 31):
        sl = slice(int(off[m]), int(off[m + 1]))
        cs = stc_lib.Context(int(off[m + 1] - off[m]), max_level=cb.max_level, **kw)
        us = cs.velocity(x[sl], z[sl], a[sl]).cpu().numpy()
        assert np.array_equal(un[sl], us), m
        cs.close()
    say(f"  {ens['steps']} RK4 steps")
    cb.rk4_batched(x, z, a, off, ens["dt"], S.OMEGA_EARTH_S, ens["steps"])
    cb.sync()
    cb.velocity_batched(x, z, a, off, out=u)
    errs = bench.ensemble_member_errors(stc_lib, x, z, a, off, u, ens["area"])
    say(f"  after stepping: worst member E = {max(errs):.3e}, median {np.median(errs):.3e}")
    assert max(errs) < 1e-6
    xh, zh, un = x.cpu().numpy(), z.cpu().numpy(), u.cpu().numpy()
    for m in range(M):
        lo, hi = int(off[m]), int(off[m + 1])
        tg = np.random.default_rng(500 + m).choice(hi - lo, 16, replace=False)
        ref = odirect.velocity(xh[lo:hi], zh[lo:hi], ens["area"][lo:hi], targets=tg, den="dist2")
        w = ens["area"][lo:hi][tg][:, None]
        e = np.sqrt((w * (un[lo:hi][tg] - ref) ** 2).sum() / (w * ref ** 2).sum())
        assert e < 2e-6, (m, e)
    cb.close()


def test_rk4_batched_matches_oracle(stc_lib):
    """Batched FP64 RK4 of a small uneven ensemble against the oracle's RK4
    through the oracle's tree code, member by member; the bar is the one the
    single-context RK4 parity test derives from the 1e-10 velocity bar."""
    from oracle import rk4 as ork4
    from oracle import tree as otree
    ens = _small_ensemble(members=3, levels=(3, 4))
    off = ens["offsets"]
    say(f"rk4 batch vs oracle N={off[-1]}")
    cb = _batched_ctx(stc_lib, ens, "fp64", "dist2")
    Om = S.OMEGA_EARTH_S
    xb, zb, ab = dev(ens["x"]), dev(ens["zeta"]), dev(ens["area"])
    cb.rk4_batched(xb, zb, ab, off, 1800.0, Om, 2)
    cb.sync()
    xg, zg = xb.cpu().numpy(), zb.cpu().numpy()
    for m in range(len(off) - 1):
        sl = slice(int(off[m]), int(off[m + 1]))
        x0, z0, a = ens["x"][sl], ens["zeta"][sl], ens["area"][sl]
        vel = lambda xx, zz, aa: otree.velocity(xx, zz, aa, max_level=cb.max_level, den="dist2", **KW)
        xr, zr = ork4.integrate(x0, z0, a, 1800.0, Om, 2, vel)
        umax = np.abs(vel(x0, z0, a)).max()
        bar_x = 1.1 * 2 * 1800.0 * 1e-10 * umax
        bar_z = 1.1 * 2 * 1800.0 * 2 * Om * 1e-10 * umax
        say(f"  member {m}: max |dx| {np.abs(xg[sl] - xr).max():.3e} (bar {bar_x:.3e})")
        assert np.abs(xg[sl] - xr).max() < bar_x
        assert np.abs(zg[sl] - zr).max() < bar_z
    cb.close()


def test_invalid_offsets_rejected(stc_lib):
    ens = _small_ensemble(members=3, levels=(3,))
    off = ens["offsets"]
    cb = _batched_ctx(stc_lib, ens, "fp64", "dot")
    x, z, a = dev(ens["x"]), dev(ens["zeta"]), dev(ens["area"])
    bad = off.copy()
    bad[1], bad[2] = bad[2], bad[1]          # decreasing
    with pytest.raises(stc_lib.StcError):
        cb.velocity_batched(x, z, a, bad)
    with pytest.raises(stc_lib.StcError):     # more members than the context holds
        cb.velocity_batched(x, z, a, np.linspace(0, off[-1], 5).astype(np.int64))
    with pytest.raises(ValueError):           # offsets must end at the row count
        cb.velocity_batched(x, z, a, off[:-1])
    cb.close()


def test_empty_member(stc_lib):
    ens = _small_ensemble(members=2, levels=(3, 4))
    off = ens["offsets"]
    off3 = np.array([0, off[1], off[1], off[2]], dtype=np.int64)   # member 1 is empty
    cb = stc_lib.Context(int(off[-1]), members=3, n_max_member=int(np.diff(off).max()), **KW)
    u = cb.velocity_batched(dev(ens["x"]), dev(ens["zeta"]), dev(ens["area"]), off3).cpu().numpy()
    for lo, hi in ((off3[0], off3[1]), (off3[2], off3[3])):
        cs = stc_lib.Context(int(hi - lo), max_level=cb.max_level, **KW)
        us = cs.velocity(dev(ens["x"][lo:hi]), dev(ens["zeta"][lo:hi]), dev(ens["area"][lo:hi])).cpu().numpy()
        assert np.array_equal(u[lo:hi], us)
        cs.close()
    cb.close()
