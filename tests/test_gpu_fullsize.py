"""GPU checks at the benchmark's full sizes, in the launch configuration
bench.py times: sampled targets against the oracle's FP64 direct sum
(computed target by target), and properties that hold at any size."""

import sys

import numpy as np
import pytest

import synthetic as S
from oracle import direct as odirect
from oracle import metrics

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _pair_coverage(ctx, n):
    """Number of ordered particle pairs (i, j), i != j, that the four lists
    cover; must be n (n - 1) for any tree and any theta.  Also checks that
    every list is strictly increasing in (target, source): the lists come out
    of the radix sort by (target, type, source) and no pair occurs twice (at
    these sizes the sort's workgroups each take several tiles)."""
    _, cnt = ctx.copy_tree()
    cnt = cnt.astype(np.int64)
    total = 0
    for kind in ("PP", "PC", "CP", "CC"):
        lst = ctx.copy_list(kind)
        t, s = lst[:, 0], lst[:, 1]
        key = (t.astype(np.int64) << 32) | s.astype(np.int64)
        assert np.all(np.diff(key) > 0), kind
        total += int((cnt[t] * cnt[s]).sum())
        if kind == "PP":
            total -= int(cnt[t[t == s]].sum())
    return total


@pytest.mark.parametrize("wl_name", ["gv_l8", "gvpair_l9"])
def test_bench_configuration_at_full_size(stc_lib, wl_name):
    import bench
    wl = S.make_workload(wl_name)
    x, z, a = wl["x"], wl["zeta"], wl["area"]
    n = len(x)
    say(f"full size {wl_name} N={n} theta={bench.BENCH_THETA} d={bench.BENCH_DEGREE}")
    xd, zd, ad = (torch.from_numpy(v).cuda() for v in (x, z, a))
    ctx = stc_lib.Context(n, theta=bench.BENCH_THETA, degree=bench.BENCH_DEGREE, n_crit=bench.BENCH_N_CRIT,
                          precision="fp32", denominator="dist2")
    u = ctx.velocity(xd, zd, ad).cpu().numpy()
    ctx.sync()
    # pair coverage holds at any size
    assert _pair_coverage(ctx, n) == n * (n - 1)
    # tangency is exact by construction (up to the final FP64 cross product)
    assert np.abs((x * u).sum(1)).max() <= 1e-12 * np.abs(u).max()
    # sampled targets against the oracle's direct sum
    idx = S.subset_indices(n, 48, 17)
    ref = odirect.velocity(x, z, a, targets=idx)
    err = metrics.rel_l2_velocity(u[idx], ref, a[idx])
    say(f"  E on 48 sampled targets vs oracle direct = {err:.3e}")
    assert err <= 1e-6
    ctx.close()


def test_fp32_and_fp64_trees_differ_by_rounding_only(stc_lib):
    """Same lists, same interpolation: the precision form differs from the
    FP64 tree code by FP32 rounding of the kernel sums only."""
    import bench
    wl = S.make_workload("gv_l8")
    x, z, a, sub = wl["x"], wl["zeta"], wl["area"], wl["subset"]
    n = len(x)
    xd, zd, ad = (torch.from_numpy(v).cuda() for v in (x, z, a))
    say("fp32 vs fp64 tree at N=655362")
    kw = dict(theta=bench.BENCH_THETA, degree=bench.BENCH_DEGREE, n_crit=bench.BENCH_N_CRIT, denominator="dist2")
    c32 = stc_lib.Context(n, precision="fp32", **kw)
    c64 = stc_lib.Context(n, precision="fp64", **kw)
    u32 = c32.velocity(xd, zd, ad).cpu().numpy()
    u64 = c64.velocity(xd, zd, ad).cpu().numpy()
    c32.close()
    c64.close()
    assert metrics.rel_l2_velocity(u32, u64, a) < 2e-7
    # and the FP64 tree against the GPU FP64 direct sum on the 4096 targets
    ud = stc_lib.direct(xd, zd, ad, targets=torch.from_numpy(sub).cuda()).cpu().numpy()
    assert metrics.rel_l2_velocity(u64[sub], ud, a[sub]) < 1e-6


def test_stream_function_at_full_size(stc_lib):
    """The stream function in the benchmark's setting at N = 655362: sampled
    targets against the oracle's direct stream function, and the GPU's FP64
    direct stream function on 48 targets against the same oracle values."""
    import bench
    wl = S.make_workload("gv_l8")
    x, z, a = wl["x"], wl["zeta"], wl["area"]
    n = len(x)
    say(f"full size stream function N={n}")
    xd, zd, ad = (torch.from_numpy(v).cuda() for v in (x, z, a))
    ctx = stc_lib.Context(n, theta=bench.BENCH_THETA, degree=bench.BENCH_DEGREE, n_crit=bench.BENCH_N_CRIT,
                          precision="fp32", denominator="dist2")
    psi = ctx.stream_function(xd, zd, ad).cpu().numpy()
    ctx.sync()
    ctx.close()
    idx = S.subset_indices(n, 48, 18)
    ref = odirect.stream_function(x, z, a, targets=idx, den="dist2")
    err = metrics.rel_l2_scalar(psi[idx], ref, a[idx])
    say(f"  E on 48 sampled targets vs oracle direct = {err:.3e}")
    assert err <= 1e-6
    dd = stc_lib.direct_stream(xd, zd, ad, targets=torch.from_numpy(idx.astype(np.int64)).cuda(),
                               denominator="dist2").cpu().numpy()
    assert np.abs(dd - ref).max() <= 1e-12 * np.abs(ref).max()


def test_forced_velocity_at_full_size(stc_lib):
    """The forced polar vortex at the paper's setting (N = 163842, d = 6,
    theta = 0.7) at full forcing, FP64 and FP32, on sampled targets against
    the oracle's direct sum of zeta - F_R (the oracle's own forcing)."""
    from oracle import forcing as oforce
    wl = S.make_workload("ssw_l7")
    x, z, a = wl["x"], wl["zeta"], wl["area"]
    n, fc, t = len(x), wl["forcing"], 8.0
    xd, zd, ad = (torch.from_numpy(v).cuda() for v in (x, z, a))
    idx = S.subset_indices(n, 48, 19)
    zf = oforce.forced_zeta(x, z, t, fc["k"], wl["omega"], fc["lat1"], fc["t_ramp"], fc["t_total"])
    ref = odirect.velocity(x, zf, a, targets=idx, den="dist2")
    for prec in ("fp64", "fp32"):
        say(f"full size forced velocity N={n} {prec}")
        ctx = stc_lib.Context(n, theta=wl["theta"], degree=wl["degree"], n_crit=64, precision=prec,
                              denominator="dist2")
        ctx.set_forcing(fc["k"], wl["omega"], fc["lat1"], fc["t_ramp"], fc["t_total"], time=t)
        u = ctx.velocity(xd, zd, ad).cpu().numpy()
        ctx.sync()
        ctx.close()
        err = metrics.rel_l2_velocity(u[idx], ref, a[idx])
        say(f"  E on 48 sampled targets vs oracle direct = {err:.3e}")
        # d = 6 at theta = 0.7 is the paper's setting, not one tuned to 1e-6:
        # the benchmark measures E = 5.3e-5 on 4096 targets
        assert err <= 2e-4
