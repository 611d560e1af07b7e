"""Pins of the oracle's adaptive mesh refinement (Appendix A) against what the
appendix and the geometry fix: hand-computed criterion values, uniform
refinement that must reproduce the icosahedral grids level by level,
coarsening back to (and never below) the initial mesh, the depth limit,
hanging midpoints, the absolute-vorticity reading for new particles, and the
quadrature weights summing to 4 pi."""

import numpy as np
import pytest

import synthetic as S
from oracle import amr


def test_criterion_hand_values():
    """The octant triangle (e_x, e_y, e_z) has area pi / 2 exactly."""
    ex, ey, ez = np.eye(3)
    A = amr.tri_area(ex, ey, ez)
    assert A == pytest.approx(np.pi / 2, rel=1e-15)
    # circulation (pi/2) * mean(zeta): mean 1 -> 1.5708; either sign counts
    assert amr.criterion(A, 1.0, 1.0, 1.0, 1.570, 10.0)
    assert not amr.criterion(A, 1.0, 1.0, 1.0, 1.571, 10.0)
    assert amr.criterion(A, -1.0, -1.0, -1.0, 1.570, 10.0)
    # the mean, not the sum: (0.5, 1, 1.5) has mean 1 as well
    assert amr.criterion(A, 0.5, 1.0, 1.5, 1.570, 10.0)
    assert not amr.criterion(A, 0.5, 1.0, 1.5, 1.571, 10.0)
    # variation max - min: 0.3
    assert amr.criterion(A, 0.0, 0.3, 0.1, 10.0, 0.3)
    assert not amr.criterion(A, 0.0, 0.3, 0.1, 10.0, 0.3000001)


def test_new_particle_carries_mean_absolute_vorticity():
    """Edge from the north pole (zeta 1) to (1, 0, 0) (zeta 3): the midpoint
    lies at z = 1/sqrt(2) and takes ((1 + 2 Om) + (3 + 0)) / 2 - 2 Om / sqrt(2)."""
    om = 0.7
    # octahedron: +z, +x, +y, -x, -y, -z
    x0 = np.array([[0, 0, 1], [1, 0, 0], [0, 1, 0], [-1, 0, 0], [0, -1, 0], [0, 0, -1]], dtype=float)
    faces = np.array([[0, 1, 2], [0, 2, 3], [0, 3, 4], [0, 4, 1], [5, 2, 1], [5, 3, 2], [5, 4, 3], [5, 1, 4]])
    m = amr.Mesh(x0, [1.0, 3.0, 0.0, 0.0, 0.0, 0.0], faces, eps1=1e9, eps2=0.5, omega=om)
    m.adapt()
    ids, x, z, a = m.particles()
    k = np.argmin(np.linalg.norm(x - np.array([1.0, 0.0, 1.0]) / np.sqrt(2.0), axis=1))
    assert np.allclose(x[k], [2 ** -0.5, 0.0, 2 ** -0.5], atol=1e-15)
    assert z[k] == pytest.approx(((1.0 + 2 * om) + 3.0) / 2 - 2 * om / np.sqrt(2.0), rel=1e-14)


@pytest.mark.parametrize("L0", [0, 1])
def test_uniform_refinement_reproduces_the_grids(L0):
    """eps2 = 0 makes every triangle meet the criterion: each pass refines all
    leaves once, so after k passes the particles are those of the icosahedral
    grid of level L0 + k (up to the depth limit 3), with the node-patch areas
    of that grid."""
    x0, f0 = S.icosahedral_grid(L0, return_faces=True)
    m = amr.Mesh(x0, np.zeros(len(x0)), f0, eps1=1e9, eps2=0.0, omega=0.0)
    for k in range(1, 5):
        m.adapt()
        _, x, _, a = m.particles()
        lvl = L0 + min(k, 3)
        xg, fg = S.icosahedral_grid(lvl, return_faces=True)
        assert len(x) == len(xg) == 10 * 4 ** lvl + 2
        # the same points (sorted by coordinates), midpoints of midpoints
        kx = np.lexsort(np.round(x, 12).T)
        kg = np.lexsort(np.round(xg, 12).T)
        assert np.abs(x[kx] - xg[kg]).max() < 1e-15
        assert np.abs(a[kx] - S.node_patch_areas(xg, fg)[kg]).max() < 1e-16
        assert a.sum() == pytest.approx(4 * np.pi, rel=1e-13)


def test_coarsening_returns_to_the_initial_mesh():
    x0, f0 = S.icosahedral_grid(1, return_faces=True)
    m = amr.Mesh(x0, np.zeros(len(x0)), f0, eps1=1e9, eps2=0.0, omega=0.0)
    for _ in range(3):
        m.adapt()
    assert len(m.particles()[0]) == 2562
    m.eps2 = 1e9                       # nothing meets the criterion any more
    counts = []
    for _ in range(4):
        m.adapt()
        counts.append(len(m.particles()[0]))
    assert counts == [642, 162, 42, 42]
    ids, x, _, a = m.particles()
    assert np.array_equal(ids, np.arange(42)) and np.array_equal(x, x0)
    assert np.abs(a - S.node_patch_areas(x0, f0)).max() < 1e-16


def test_local_refinement_hanging_midpoints_and_depth_limit():
    """One strong vortex particle: only the triangles around it are split,
    down to three levels and no further; every live particle is a vertex of a
    leaf, midpoints on a split triangle's edges next to an unsplit neighbour
    take area from the split side only, and the areas still sum to 4 pi."""
    x0, f0 = S.icosahedral_grid(2, return_faces=True)
    z0 = np.zeros(len(x0))
    z0[37] = 10.0
    m = amr.Mesh(x0, z0, f0, eps1=1e9, eps2=1.0, omega=0.0)
    sizes = []
    for _ in range(5):
        m.adapt()
        sizes.append(len(m.particles()[0]))
    # the 5 or 6 triangles around particle 37 split; later passes split the
    # children that still touch it; the counts stop growing at depth 3
    assert sizes[0] > len(x0) and sizes[1] > sizes[0] and sizes[2] > sizes[1]
    assert sizes[3] == sizes[2] == sizes[4]
    assert max(m.depth[t] for t in m.leaves()) == 3
    ids, x, z, a = m.particles()
    assert a.sum() == pytest.approx(4 * np.pi, rel=1e-13)
    used = set()
    for t in m.leaves():
        used.update(m.tv[t])
    assert used == set(ids.tolist())
    # vorticity interpolated from the field: new particles have 0 <= zeta <= 10
    assert (z >= 0).all() and (z <= 10.0).all()


def test_gaussian_vortex_initial_resolution():
    """The Gaussian-vortex configuration (eps1 = 0.0025, eps2 = 0.2, 10242
    initial particles): resolving the initial field refines around the
    vortex only, by at most three levels, keeps every initial particle and
    stays below the about 36000 particles the paper's runs end with after
    three days (the vortex's filament adds more); C keeps the total
    vorticity zero."""
    x0, f0 = S.icosahedral_grid(5, return_faces=True)
    a0 = S.node_patch_areas(x0, f0)
    m = amr.Mesh(x0, S.gaussian_vortex_paper(x0, a0), f0, eps1=0.0025, eps2=0.2, omega=2 * np.pi)

    def zeta_fn(x):
        _, _, _, a = m.particles()
        return S.gaussian_vortex_paper(x, a)

    m.resolve_initial(zeta_fn)
    ids, x, z, a = m.particles()
    assert set(range(len(x0))) <= set(ids.tolist())
    assert 20000 < len(ids) < 36000
    assert abs((z * a).sum()) < 1e-12
    xc = np.array([np.cos(np.pi / 20), 0.0, np.sin(np.pi / 20)])
    new = x[len(x0):]
    assert np.linalg.norm(new - xc, axis=1).max() < 1.0     # added particles sit near the vortex


def test_areas_are_carried_not_recomputed():
    """Moving the particles changes no weight: the triangles carry their
    areas (the flow is incompressible); a split shares the parent's carried
    area among its children in proportion to their spherical areas, so the
    weights still sum to 4 pi even when the particles have moved; a merge
    gives the parent its own carried area back."""
    x0, f0 = S.icosahedral_grid(1, return_faces=True)
    z0 = np.zeros(len(x0))
    m = amr.Mesh(x0, z0, f0, eps1=1e9, eps2=0.5, omega=0.0)
    a0 = m.particles()[3].copy()
    # move every particle (a rotation plus a perturbation): no pass, no change of weights
    rng = np.random.default_rng(3)
    R = S.random_rotation(9)
    xm = x0 @ R.T + 0.02 * rng.standard_normal(x0.shape)
    xm /= np.linalg.norm(xm, axis=1, keepdims=True)
    m.set_state(np.arange(len(x0)), xm, z0)
    assert np.array_equal(m.particles()[3], a0)
    # a spread of 1 at one particle splits its triangles there
    z1 = z0.copy()
    z1[7] = 1.0
    m.set_state(np.arange(len(x0)), xm, z1)
    m.adapt()
    ids, x, z, a = m.particles()
    assert len(ids) > len(x0)
    assert a.sum() == pytest.approx(4 * np.pi, rel=1e-13)
    # every split triangle's children carry exactly its area between them
    for t in range(len(m.tv)):
        if m.state[t] == amr.REFINED:
            ch = m.children[t]
            assert sum(m.tarea[c] for c in ch) == pytest.approx(m.tarea[t], rel=1e-14)
    # merge back: the initial weights return bitwise
    m.set_state(ids, x, np.zeros(len(ids)))
    m.adapt()
    assert np.array_equal(m.particles()[3], a0)
