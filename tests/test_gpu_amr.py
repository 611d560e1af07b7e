"""GPU adaptive mesh refinement (Appendix A) against the oracle's, through the
C ABI.  Particles are matched by identity: an initial particle by its index,
a midpoint by the unordered pair of its edge ends' identities (the library
reports each particle slot's edge ends, the oracle its edge dictionary), so
the comparison does not depend on either side's numbering.

Bars: the live particle sets identical after every pass; positions and
vorticities of the adapted mesh bitwise equal (the same formulas in the same
order; contraction off); areas within 1e-15 relative (the arctangent of the
two sides may differ in its last bit); with time steps in between, the sets
identical and the states within the RK4 parity bars.
"""

import sys

import numpy as np
import pytest

import synthetic as S
from oracle import amr as oamr
from oracle import rk4 as ork4
from oracle import tree as otree

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_ids(mesh, n0):
    slots, ends = mesh.slots()
    memo = {}

    def ident(v):
        if v < n0:
            return (int(v),)
        if v not in memo:
            a, b = ends[v]
            memo[v] = frozenset((ident(a), ident(b)))
        return memo[v]

    return [ident(int(v)) for v in slots]


def oracle_ids(m, n0):
    ends = {v: k for k, v in m.edge_mid.items()}
    memo = {}

    def ident(v):
        if v < n0:
            return (int(v),)
        if v not in memo:
            a, b = ends[v]
            memo[v] = frozenset((ident(a), ident(b)))
        return memo[v]

    ids = m.particles()[0]
    return [ident(int(v)) for v in ids]


def compare(mesh, m, n0, exact=True, tol_x=0.0, tol_z=0.0, tol_a=1e-15):
    gi = gpu_ids(mesh, n0)
    oi = oracle_ids(m, n0)
    assert len(gi) == len(oi) and set(gi) == set(oi)
    pos = {k: j for j, k in enumerate(oi)}
    perm = np.array([pos[k] for k in gi])
    x, z, a = (t.cpu().numpy() for t in mesh.particles())
    _, xo, zo, ao = m.particles()
    xo, zo, ao = xo[perm], zo[perm], ao[perm]
    if exact:
        assert np.array_equal(x, xo) and np.array_equal(z, zo)
    else:
        assert np.abs(x - xo).max() <= tol_x
        assert np.abs(z - zo).max() <= tol_z * np.abs(zo).max()
    assert np.abs(a - ao).max() <= tol_a * np.abs(ao).max()
    return len(gi)


def test_uniform_refinement_and_coarsening(stc_lib):
    """zeta = 1 everywhere with eps1 below every triangle's area: each pass
    splits all leaves (L1 -> L4 particle counts, then the depth limit); zeta
    set to 0 at every live particle: each pass merges one level, back to the
    initial mesh and no further."""
    x0, f0 = S.icosahedral_grid(1, return_faces=True)
    z0 = np.ones(len(x0))
    mesh = stc_lib.AdaptiveMesh(x0, f0, eps1=1e-6, eps2=1e9, omega=0.0)
    mesh.set_state(dev(x0), dev(z0))
    m = oamr.Mesh(x0, z0, f0, eps1=1e-6, eps2=1e9, omega=0.0)
    counts = []
    for k in range(4):
        say(f"uniform refinement pass {k}")
        mesh.adapt()
        m.adapt()
        counts.append(compare(mesh, m, len(x0)))
    assert counts == [162, 642, 2562, 2562]
    assert mesh.stats()["capacity"] == 2562
    x, z, _ = mesh.particles()
    mesh.set_state(x.clone(), torch.zeros_like(z))
    ids, xo, _, _ = m.particles()
    m.set_state(ids, xo, np.zeros(len(ids)))
    counts = []
    for k in range(4):
        say(f"coarsening pass {k}")
        mesh.adapt()
        m.adapt()
        counts.append(compare(mesh, m, len(x0)))
    assert counts == [642, 162, 42, 42]
    x, _, a = mesh.particles()
    assert np.array_equal(x.cpu().numpy(), x0)
    assert np.abs(a.cpu().numpy() - S.node_patch_areas(x0, f0)).max() < 1e-16
    mesh.close()


@pytest.mark.parametrize("L0,eps1,eps2", [(2, 0.02, 0.5), (3, 0.0025, 0.2)])
def test_gaussian_vortex_passes_match_oracle(stc_lib, L0, eps1, eps2):
    """The Gaussian vortex of Sec. 4.3 on a coarse initial mesh: five passes,
    the new particles' vorticity from the interpolation reading; the leaf
    counts of the two sides agree as well."""
    x0, f0 = S.icosahedral_grid(L0, return_faces=True)
    a0 = S.node_patch_areas(x0, f0)
    z0 = S.gaussian_vortex_paper(x0, a0)
    om = S.OMEGA_EARTH_DAY
    mesh = stc_lib.AdaptiveMesh(x0, f0, eps1=eps1, eps2=eps2, omega=om)
    mesh.set_state(dev(x0), dev(z0))
    m = oamr.Mesh(x0, z0, f0, eps1=eps1, eps2=eps2, omega=om)
    sizes = []
    for k in range(5):
        mesh.adapt()
        m.adapt()
        sizes.append(compare(mesh, m, len(x0)))
        say(f"L0={L0} pass {k}: {sizes[-1]} particles")
    assert sizes[0] > len(x0)
    st = mesh.stats()
    assert st["leaves"] == len(m.leaves())
    mesh.close()


def test_rk4_with_adaptation_matches_oracle(stc_lib):
    """Initial mesh L2 (162 particles), Gaussian vortex, AMR thresholds that
    refine around the vortex; three RK4 steps of 0.01 day with a pass after
    each, against the oracle's RK4 through its tree code and its passes.
    Bars: the RK4 parity bars (2 dt 1e-10 max|u| per step) on positions and
    vorticities; identical particle sets."""
    x0, f0 = S.icosahedral_grid(2, return_faces=True)
    a0 = S.node_patch_areas(x0, f0)
    z0 = S.gaussian_vortex_paper(x0, a0)
    om, dt, eps1, eps2 = S.OMEGA_EARTH_DAY, 0.01, 0.02, 0.5
    kw = dict(theta=0.7, degree=6, n_crit=16)
    mesh = stc_lib.AdaptiveMesh(x0, f0, eps1=eps1, eps2=eps2, omega=om)
    mesh.set_state(dev(x0), dev(z0))
    m = oamr.Mesh(x0, z0, f0, eps1=eps1, eps2=eps2, omega=om)
    mesh.adapt()
    m.adapt()
    compare(mesh, m, len(x0))
    cap = mesh.stats()["capacity"]
    ctx = stc_lib.Context(cap, max_level=4, denominator="dist2", **kw)
    vel = lambda xx, zz, aa: otree.velocity(xx, zz, aa, max_level=4, den="dist2", **kw)
    for step in range(3):
        say(f"rk4 + amr step {step}")
        _, xo, zo, ao = m.particles()
        umax = np.abs(vel(xo, zo, ao)).max()
        mesh.rk4(ctx, dt, om, 1)
        oamr.step_with_amr(m, dt, vel, ork4.step)
        compare(mesh, m, len(x0), exact=False, tol_x=1.1 * 2 * dt * 1e-10 * umax * (step + 1),
                tol_z=1e-9, tol_a=1e-9)
    ctx.close()
    mesh.close()
