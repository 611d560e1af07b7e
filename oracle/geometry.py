"""Triangle tree geometry and exact point location.  TEST INFRASTRUCTURE ONLY.

The tree (Sec. 3, overview and grids) starts from the 20 faces of an
icosahedron and splits every face into four, level by level.  Readings used
where the paper is silent:

* Icosahedron: unnormalised vertices (0,+-1,+-phi), (+-1,+-phi,0),
  (+-phi,0,+-1) in lexicographic (x, y, z) order, normalised as
  p / sqrt((px*px + py*py) + pz*pz).  Faces: mutually adjacent triples
  i < j < k, lexicographic, stored counter-clockwise seen from outside.
* Children of (v1, v2, v3): 0 = (v1, m12, m31), 1 = (m12, v2, m23),
  2 = (m31, m23, v3), 3 = (m12, m23, m31), m_ab = (a + b) / |a + b|.
* Node (level l, key k): k = face * 4^l + sum of child digits; its global id
  is 20 (4^l - 1) / 3 + k.
* Circumcentre c = normalise((v2 - v1) x (v3 - v1)); radius r = the largest
  chord |c - v_k| (Sec. 3, dual tree traversal: radii and circumcentres).
* Point location uses the exact sign of det[a, b, p] = p . (a x b): a
  floating-point filter with a proven error bound, and exact rational
  arithmetic (``fractions.Fraction``) when the filter cannot decide.
  Root face: the lowest face index whose three edge orientations are all
  >= 0.  Child: corner 1, 2, 3 if p lies strictly outside the centre child
  across the edge facing that corner (tested in that order), else the centre.

All decision geometry uses IEEE +, -, *, /, sqrt in the order written, so
another implementation of the same recipe reaches bitwise identical values.
"""

from fractions import Fraction

import numpy as np

PHI = (1.0 + 5.0 ** 0.5) / 2.0
EPS = 2.0 ** -53


def level_offset(level):
    return 20 * (4 ** level - 1) // 3


def total_nodes(max_level):
    return level_offset(max_level + 1)


def node_level_key(node_id):
    lvl = 0
    while level_offset(lvl + 1) <= node_id:
        lvl += 1
    return lvl, node_id - level_offset(lvl)


def _normalize(p):
    n = np.sqrt((p[..., 0] * p[..., 0] + p[..., 1] * p[..., 1]) + p[..., 2] * p[..., 2])
    return p / n[..., None]


def base_icosahedron():
    raw = sorted({(0.0, s1, s2 * PHI) for s1 in (-1.0, 1.0) for s2 in (-1.0, 1.0)}
                 | {(s1, s2 * PHI, 0.0) for s1 in (-1.0, 1.0) for s2 in (-1.0, 1.0)}
                 | {(s2 * PHI, 0.0, s1) for s1 in (-1.0, 1.0) for s2 in (-1.0, 1.0)})
    raw = np.array(raw)
    verts = _normalize(raw)
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            for k in range(j + 1, 12):
                dij = ((raw[i] - raw[j]) ** 2).sum()
                dik = ((raw[i] - raw[k]) ** 2).sum()
                djk = ((raw[j] - raw[k]) ** 2).sum()
                if abs(dij - 4) < 1e-9 and abs(dik - 4) < 1e-9 and abs(djk - 4) < 1e-9:
                    orient = np.dot(np.cross(raw[j] - raw[i], raw[k] - raw[i]), raw[i])
                    faces.append((i, j, k) if orient > 0 else (i, k, j))
    return verts, faces


class TreeGeometry:
    """Vertices, circumcentres and radii of every node down to max_level."""

    def __init__(self, max_level):
        self.max_level = max_level
        verts, faces = base_icosahedron()
        v = np.array([[verts[a], verts[b], verts[c]] for a, b, c in faces])
        self.verts = [v]                       # per level: (20*4^l, 3, 3)
        for _ in range(max_level):
            p = self.verts[-1]
            v1, v2, v3 = p[:, 0], p[:, 1], p[:, 2]
            m12 = _normalize(v1 + v2)
            m23 = _normalize(v2 + v3)
            m31 = _normalize(v3 + v1)
            ch = np.stack([np.stack([v1, m12, m31], 1),
                           np.stack([m12, v2, m23], 1),
                           np.stack([m31, m23, v3], 1),
                           np.stack([m12, m23, m31], 1)], 1)
            self.verts.append(ch.reshape(-1, 3, 3))
        self.center = []
        self.radius = []
        for v in self.verts:
            e1 = v[:, 1] - v[:, 0]
            e2 = v[:, 2] - v[:, 0]
            cr = np.stack([e1[:, 1] * e2[:, 2] - e1[:, 2] * e2[:, 1],
                           e1[:, 2] * e2[:, 0] - e1[:, 0] * e2[:, 2],
                           e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]], 1)
            c = _normalize(cr)
            r = None
            for k in range(3):
                d = c - v[:, k]
                rk = np.sqrt((d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2])
                r = rk if r is None else np.maximum(r, rk)
            self.center.append(c)
            self.radius.append(r)

    def node_vertices(self, node_id):
        lvl, key = node_level_key(node_id)
        return self.verts[lvl][key]

    def node_center(self, node_id):
        lvl, key = node_level_key(node_id)
        return self.center[lvl][key]

    def node_radius(self, node_id):
        lvl, key = node_level_key(node_id)
        return float(self.radius[lvl][key])


# --- exact orientation -------------------------------------------------------

def _orient_exact(a, b, p):
    ax, ay, az = (Fraction(float(t)) for t in a)
    bx, by, bz = (Fraction(float(t)) for t in b)
    px, py, pz = (Fraction(float(t)) for t in p)
    det = px * (ay * bz - az * by) + py * (az * bx - ax * bz) + pz * (ax * by - ay * bx)
    return (det > 0) - (det < 0)


def orient(a, b, p):
    """Exact sign of p . (a x b) for rows of (M, 3) arrays a, b, p -> int8 (M,)."""
    cx = a[:, 1] * b[:, 2] - a[:, 2] * b[:, 1]
    cy = a[:, 2] * b[:, 0] - a[:, 0] * b[:, 2]
    cz = a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]
    det = (p[:, 0] * cx + p[:, 1] * cy) + p[:, 2] * cz
    perm = (np.abs(p[:, 0]) * (np.abs(a[:, 1] * b[:, 2]) + np.abs(a[:, 2] * b[:, 1]))
            + np.abs(p[:, 1]) * (np.abs(a[:, 2] * b[:, 0]) + np.abs(a[:, 0] * b[:, 2]))
            + np.abs(p[:, 2]) * (np.abs(a[:, 0] * b[:, 1]) + np.abs(a[:, 1] * b[:, 0])))
    # the rounding error of `det` is at most ~5 eps * perm; 8 eps is safe
    bound = 8.0 * EPS * perm
    out = np.sign(det).astype(np.int8)
    unsure = np.nonzero(~(np.abs(det) > bound))[0]
    for i in unsure:
        out[i] = _orient_exact(a[i], b[i], p[i])
    return out


def locate(x, geom):
    """Leaf key at geom.max_level for every point (exact point location)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    L = geom.max_level
    root = geom.verts[0]
    face = np.full(n, -1, dtype=np.int64)
    for f in range(20):
        todo = np.nonzero(face < 0)[0]
        if len(todo) == 0:
            break
        p = x[todo]
        v1 = np.broadcast_to(root[f, 0], p.shape)
        v2 = np.broadcast_to(root[f, 1], p.shape)
        v3 = np.broadcast_to(root[f, 2], p.shape)
        ok = (orient(v1, v2, p) >= 0) & (orient(v2, v3, p) >= 0) & (orient(v3, v1, p) >= 0)
        face[todo[ok]] = f
    assert (face >= 0).all(), "point outside every face"
    key = face.copy()
    for lvl in range(L):
        centre_child = geom.verts[lvl + 1][4 * key + 3]   # (m12, m23, m31)
        m12, m23, m31 = centre_child[:, 0], centre_child[:, 1], centre_child[:, 2]
        c1 = orient(m31, m12, x) < 0
        c2 = orient(m12, m23, x) < 0
        c3 = orient(m23, m31, x) < 0
        digit = np.where(c1, 0, np.where(c2, 1, np.where(c3, 2, 3)))
        key = 4 * key + digit
    return key


class ParticleTree:
    """Particles binned into the tree: permutation, per-node ranges, counts."""

    def __init__(self, x, geom, n_crit):
        self.geom = geom
        self.n_crit = n_crit
        L = geom.max_level
        self.leaf_key = locate(x, geom)
        # sorted order: by leaf key, ties by original index
        self.perm = np.argsort(self.leaf_key, kind="stable")
        sk = self.leaf_key[self.perm]
        self.count = np.zeros(total_nodes(L), dtype=np.int64)
        self.begin = np.zeros(total_nodes(L), dtype=np.int64)
        for lvl in range(L + 1):
            pref = sk >> (2 * (L - lvl))
            nl = 20 * 4 ** lvl
            cnt = np.bincount(pref, minlength=nl)
            off = level_offset(lvl)
            self.count[off:off + nl] = cnt
            self.begin[off:off + nl] = np.concatenate([[0], np.cumsum(cnt)[:-1]])

    def level(self, node_id):
        return node_level_key(node_id)[0]

    def is_internal(self, node_id):
        return self.count[node_id] > self.n_crit and self.level(node_id) < self.geom.max_level

    def children(self, node_id):
        lvl, key = node_level_key(node_id)
        off = level_offset(lvl + 1)
        return [off + 4 * key + c for c in range(4)]

    def members(self, node_id):
        b = self.begin[node_id]
        return self.perm[b:b + self.count[node_id]]
