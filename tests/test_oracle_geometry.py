"""Pins for the oracle's tree geometry, exact predicates and point location."""

from fractions import Fraction

import numpy as np
import pytest

import synthetic as S
from oracle import geometry as G
from oracle import tree as T


def test_icosahedron_faces_ccw_and_closed():
    verts, faces = G.base_icosahedron()
    assert len(verts) == 12 and len(faces) == 20
    np.testing.assert_allclose(np.linalg.norm(verts, axis=1), 1.0, atol=1e-15)
    edges = {}
    for f in faces:
        a, b, c = (verts[i] for i in f)
        assert np.dot(np.cross(b - a, c - a), a) > 0
        for e in ((f[0], f[1]), (f[1], f[2]), (f[2], f[0])):
            edges[tuple(sorted(e))] = edges.get(tuple(sorted(e)), 0) + 1
    assert len(edges) == 30 and set(edges.values()) == {2}
    # the generator's icosahedron is the same point set, same order
    np.testing.assert_array_equal(verts, S.icosahedron_vertices())


def test_level0_radius_closed_form():
    """Chord from a face's circumcentre to its vertices: cos(a) = phi^2 /
    (sqrt(3) sqrt(1 + phi^2)) (inradius over circumradius of the icosahedron)."""
    geom = G.TreeGeometry(0)
    phi = (1 + 5 ** 0.5) / 2
    cos_a = phi ** 2 / (3 ** 0.5 * (1 + phi ** 2) ** 0.5)
    chord = (2 - 2 * cos_a) ** 0.5
    np.testing.assert_allclose(geom.radius[0], chord, rtol=1e-14)
    assert abs(chord - 0.64085) < 1e-5


def test_level0_mac_ratios_and_separated_pairs():
    """Face centres are dodecahedron vertices: the cosines between them are
    1, sqrt5/3 (x3), 1/3 (x6), -1/3 (x6), -sqrt5/3 (x3), -1.  At theta = 0.7
    exactly the antipodal and the three next-farthest faces are separated:
    80 of the 400 root pairs."""
    geom = G.TreeGeometry(0)
    c = geom.center[0]
    cosines = np.sort(np.round(c @ c.T, 12), axis=1)
    s5 = 5 ** 0.5 / 3
    expect = np.sort(np.round([1, s5, s5, s5, 1 / 3] + [1 / 3] * 5 + [-1 / 3] * 6
                              + [-s5] * 3 + [-1], 12))
    for row in cosines:
        np.testing.assert_allclose(row, expect, atol=1e-12)
    sep = sum(T.well_separated(geom, t, s, 0.7) for t in range(20) for s in range(20))
    assert sep == 80
    r = geom.radius[0][0]
    for cs, ratio in ((-1, 0.6409), (-s5, 0.686), (-1 / 3, 0.785), (1 / 3, 1.11), (s5, 1.80)):
        R = (2 - 2 * cs) ** 0.5
        assert abs(2 * r / R - ratio) < 5e-3


def _orient_fraction(a, b, p):
    a = [Fraction(float(v)) for v in a]
    b = [Fraction(float(v)) for v in b]
    p = [Fraction(float(v)) for v in p]
    det = (p[0] * (a[1] * b[2] - a[2] * b[1]) + p[1] * (a[2] * b[0] - a[0] * b[2])
           + p[2] * (a[0] * b[1] - a[1] * b[0]))
    return (det > 0) - (det < 0)


def test_orient_is_exact_on_degenerate_inputs():
    rng = np.random.default_rng(0)
    a = S.random_sphere_points(300, 1)
    b = S.random_sphere_points(300, 2)
    # points on, or within a few ulps of, the great circle through a and b
    t = rng.random(300)
    p = t[:, None] * a + (1 - t[:, None]) * b
    p = p / np.linalg.norm(p, axis=1)[:, None]
    p[:100] += rng.integers(-2, 3, (100, 3)) * np.spacing(p[:100])
    p[100:110] = a[100:110]
    p[110:120] = -b[110:120]
    got = G.orient(a, b, p)
    want = np.array([_orient_fraction(a[i], b[i], p[i]) for i in range(300)])
    np.testing.assert_array_equal(got, want)
    assert (want == 0).sum() >= 20
    np.testing.assert_array_equal(G.orient(b, a, p), -want)


@pytest.mark.parametrize("pts", ["grid", "random"])
def test_locate_places_points_in_their_leaf(pts):
    L = 3
    geom = G.TreeGeometry(L)
    x = S.icosahedral_grid(3) if pts == "grid" else S.random_sphere_points(2000, 4)
    key = G.locate(x, geom)
    tri = geom.verts[L][key]
    for k in range(3):
        a, b = tri[:, k], tri[:, (k + 1) % 3]
        # every point lies in its closed leaf triangle (exactly, or within
        # rounding of the refined edges for points that sit on an edge)
        o = np.einsum("ij,ij->i", x, np.cross(a, b))
        assert (o > -1e-15).all()
    counts = np.bincount(key, minlength=20 * 4 ** L)
    assert counts.sum() == len(x)


def test_grid_points_on_edges_use_tie_rule():
    """Every unrotated grid point sits on tree edges; the exact predicates
    and the tie rule still give one leaf per point, and the counts are
    nested level by level."""
    x = S.icosahedral_grid(4)
    geom = G.TreeGeometry(4)
    pt = G.ParticleTree(x, geom, n_crit=8)
    for lvl in range(4):
        off, off1 = G.level_offset(lvl), G.level_offset(lvl + 1)
        nl = 20 * 4 ** lvl
        parent = pt.count[off:off + nl]
        kids = pt.count[off1:off1 + 4 * nl].reshape(nl, 4).sum(1)
        np.testing.assert_array_equal(parent, kids)
    assert pt.count[:20].sum() == len(x)
    # permutation is a stable sort by leaf key
    assert (np.diff(pt.leaf_key[pt.perm]) >= 0).all()
