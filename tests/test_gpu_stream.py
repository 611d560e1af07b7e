"""GPU stream function (Sec. 2, stream function; the logarithmic kernel through
the same tree, Sec. 3) against the oracle: the direct sum (one chunk and
split into source chunks), the tree code in FP64 with both denominators on
grid, rotated-grid and ragged random inputs, and the FP32 form."""

import sys

import numpy as np
import pytest

import synthetic as S
from oracle import direct as odirect
from oracle import tree as otree

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("den", ["dot", "dist2"])
def test_direct_stream_matches_oracle(stc_lib, den):
    x = S.icosahedral_grid(4) @ S.random_rotation(31).T
    z = S.rossby_haurwitz(x, 4)
    a = S.uniform_areas(len(x))
    say(f"direct stream all targets N={len(x)} {den}")
    got = stc_lib.direct_stream(dev(x), dev(z), dev(a), denominator=den).cpu().numpy()
    ref = odirect.stream_function(x, z, a, den=den)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_direct_stream_split_sources(stc_lib):
    """Few targets and many sources: the sum runs in source chunks reduced in
    a fixed order."""
    x = S.icosahedral_grid(6)
    z = S.gaussian_vortex(x, seed=3)
    a = S.uniform_areas(len(x))
    sub = S.subset_indices(len(x), 96, 3)
    say(f"direct stream 96 targets x {len(x)} sources")
    got = stc_lib.direct_stream(dev(x), dev(z), dev(a), targets=dev(sub.astype(np.int64))).cpu().numpy()
    ref = odirect.stream_function(x, z, a, targets=sub)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    f32 = stc_lib.direct_stream(dev(x), dev(z), dev(a), targets=dev(sub.astype(np.int64)), precision="fp32",
                                denominator="dist2").cpu().numpy()
    assert np.abs(f32 - ref).max() <= 1e-5 * np.abs(ref).max()


CASES = {
    "rotated_l4": lambda: (S.icosahedral_grid(4) @ S.random_rotation(32).T, 4),
    "grid_l4": lambda: (S.icosahedral_grid(4), 4),
    "random_7001": lambda: (S.random_sphere_points(7001, 5), 5),
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("den", ["dot", "dist2"])
def test_tree_stream_fp64_matches_oracle_tree(stc_lib, name, den):
    x, L = CASES[name]()
    z = S.rossby_haurwitz(x, 3)
    a = S.uniform_areas(len(x))
    th, d, nc = 0.7, 6, 32
    say(f"tree stream fp64 {name} {den} N={len(x)}")
    ctx = stc_lib.Context(len(x), theta=th, degree=d, n_crit=nc, max_level=L, denominator=den)
    got = ctx.stream_function(dev(x), dev(z), dev(a)).cpu().numpy()
    ctx.sync()
    ot = otree.TreeCode(x, z, a, theta=th, degree=d, n_crit=nc, max_level=L, den=den,
                        kernel=otree.stream_kernel(den))
    ref = ot.stream_function()
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-10 * scale
    # a velocity after the stream function is bitwise the one of a fresh context
    u = ctx.velocity(dev(x), dev(z), dev(a))
    fresh = stc_lib.Context(len(x), theta=th, degree=d, n_crit=nc, max_level=L, denominator=den)
    assert torch.equal(u, fresh.velocity(dev(x), dev(z), dev(a)))
    fresh.close()
    ctx.close()


def test_tree_stream_fp32_and_accuracy_against_direct(stc_lib):
    x = S.icosahedral_grid(5) @ S.random_rotation(33).T
    z = S.gaussian_vortex(x, seed=4)
    a = S.uniform_areas(len(x))
    say(f"tree stream fp32 vs fp64 vs direct N={len(x)}")
    exact = odirect.stream_function(x, z, a, den="dist2")
    scale = np.abs(exact).max()
    c64 = stc_lib.Context(len(x), theta=0.7, degree=8, n_crit=64, denominator="dist2")
    c32 = stc_lib.Context(len(x), theta=0.7, degree=8, n_crit=64, precision="fp32", denominator="dist2")
    p64 = c64.stream_function(dev(x), dev(z), dev(a)).cpu().numpy()
    p32 = c32.stream_function(dev(x), dev(z), dev(a)).cpu().numpy()
    assert np.abs(p64 - exact).max() <= 1e-4 * scale
    assert np.abs(p32 - p64).max() <= 1e-5 * scale
    c64.close()
    c32.close()


@pytest.mark.parametrize("precision,den", [("fp64", "dot"), ("fp32", "dist2")])
def test_stream_function_batched_bitwise_equal_single(stc_lib, precision, den):
    """Ensembles: every member's stream function equals a single-member
    context's, bitwise; members of a few sizes and rotations."""
    ens = S.make_ensemble(members=4, seed0=4, levels=(3, 4, 5))
    off = ens["offsets"]
    kw = dict(theta=0.7, degree=6, n_crit=32, precision=precision, denominator=den)
    say(f"batched stream function {len(off) - 1} members N={off[-1]} {precision} {den}")
    cb = stc_lib.Context(int(off[-1]), members=len(off) - 1, n_max_member=int(np.diff(off).max()), **kw)
    psi = cb.stream_function_batched(dev(ens["x"]), dev(ens["zeta"]), dev(ens["area"]), off)
    cb.sync()
    for m in range(len(off) - 1):
        sl = slice(off[m], off[m + 1])
        cs = stc_lib.Context(int(off[m + 1] - off[m]), max_level=cb.max_level, **kw)
        ps = cs.stream_function(dev(ens["x"][sl]), dev(ens["zeta"][sl]), dev(ens["area"][sl]))
        assert torch.equal(psi[sl], ps), m
        cs.close()
    cb.close()
