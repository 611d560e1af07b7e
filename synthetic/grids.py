"""Particle sets and quadrature weights (Sec. 2: refined-icosahedron particles,
node-patch areas).

The base icosahedron uses the unnormalised vertices (0, +-1, +-phi),
(+-1, +-phi, 0), (+-phi, 0, +-1), ordered lexicographically by (x, y, z), each
normalised as p / sqrt(px*px + py*py + pz*pz).  Faces are the mutually adjacent
vertex triples i < j < k in lexicographic order, stored counter-clockwise seen
from outside.  Refinement splits a face (v1, v2, v3) into (v1, m12, m31),
(m12, v2, m23), (m31, m23, v3), (m12, m23, m31) with m_ab = (a + b) / |a + b|.
Every operation is an elementwise IEEE operation in a fixed order, so a grid
vertex is bit-for-bit the point any other code computes with the same recipe.
"""

import numpy as np

PHI = (1.0 + np.sqrt(5.0)) / 2.0


def _normalize_rows(p):
    # elementwise, left-to-right: (x*x + y*y) + z*z, then sqrt, then divide
    n = np.sqrt((p[:, 0] * p[:, 0] + p[:, 1] * p[:, 1]) + p[:, 2] * p[:, 2])
    return p / n[:, None]


def icosahedron_vertices(normalized=True):
    raw = []
    for a in (-1.0, 1.0):
        for b in (-PHI, PHI):
            raw.append((0.0, a, b))
            raw.append((a, b, 0.0))
            raw.append((b, 0.0, a))
    raw.sort()
    p = np.array(raw, dtype=np.float64)
    return _normalize_rows(p) if normalized else p


def icosahedron_faces():
    raw = icosahedron_vertices(normalized=False)
    n = len(raw)
    d2 = ((raw[:, None, :] - raw[None, :, :]) ** 2).sum(-1)
    adj = np.isclose(d2, 4.0)
    faces = []
    for i in range(n):
        for j in range(i + 1, n):
            if not adj[i, j]:
                continue
            for k in range(j + 1, n):
                if adj[i, k] and adj[j, k]:
                    e1 = raw[j] - raw[i]
                    e2 = raw[k] - raw[i]
                    if np.dot(np.cross(e1, e2), raw[i]) > 0:
                        faces.append((i, j, k))
                    else:
                        faces.append((i, k, j))
    assert len(faces) == 20
    return np.array(faces, dtype=np.int64)


def grid_size(level):
    """Number of vertices of the icosahedron refined `level` times."""
    return 10 * 4 ** level + 2


def icosahedral_grid(level, return_faces=False):
    """Vertices (N, 3) of the icosahedron refined `level` times (N = 10*4^L+2).

    Vertex order: the 12 base vertices, then at each refinement the new edge
    midpoints in increasing order of their (min, max) parent-vertex pair.
    """
    verts = icosahedron_vertices()
    faces = icosahedron_faces()
    for _ in range(level):
        nv = len(verts)
        a, b, c = faces[:, 0], faces[:, 1], faces[:, 2]
        edges = np.concatenate([np.stack([a, b], 1), np.stack([b, c], 1),
                                np.stack([c, a], 1)])
        lo = edges.min(1)
        hi = edges.max(1)
        code = lo * nv + hi
        uniq, inv = np.unique(code, return_inverse=True)
        ulo = uniq // nv
        uhi = uniq % nv
        s = verts[ulo] + verts[uhi]
        mids = _normalize_rows(s)
        mid_index = nv + inv
        nf = len(faces)
        m_ab = mid_index[:nf]
        m_bc = mid_index[nf:2 * nf]
        m_ca = mid_index[2 * nf:]
        children = np.stack([
            np.stack([a, m_ab, m_ca], 1),
            np.stack([m_ab, b, m_bc], 1),
            np.stack([m_ca, m_bc, c], 1),
            np.stack([m_ab, m_bc, m_ca], 1),
        ], 1).reshape(-1, 3)
        verts = np.concatenate([verts, mids])
        faces = children
    if return_faces:
        return verts, faces
    return verts


def uniform_areas(n):
    """A_j = 4 pi / N for every particle."""
    return np.full(n, 4.0 * np.pi / n, dtype=np.float64)


def _spherical_triangle_area(a, b, c):
    # Van Oosterom & Strackee (1983): tan(E/2) = |a.(b x c)| / (1 + a.b + b.c + c.a)
    trip = np.abs(np.einsum("ij,ij->i", a, np.cross(b, c)))
    den = 1.0 + np.einsum("ij,ij->i", a, b) + np.einsum("ij,ij->i", b, c) \
        + np.einsum("ij,ij->i", c, a)
    return 2.0 * np.arctan2(trip, den)


def node_patch_areas(verts, faces):
    """Node-patch (barycentric dual) areas: A_i = sum over faces touching i of
    area(face) / 3.  They sum to 4 pi."""
    area = _spherical_triangle_area(verts[faces[:, 0]], verts[faces[:, 1]],
                                    verts[faces[:, 2]])
    out = np.zeros(len(verts))
    for k in range(3):
        np.add.at(out, faces[:, k], area / 3.0)
    return out


def random_rotation(seed):
    """Uniform random rotation (QR of a Gaussian 3x3 with sign fix, det +1)."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def random_sphere_points(n, seed):
    """n points uniformly distributed on the unit sphere."""
    rng = np.random.default_rng(seed)
    p = rng.standard_normal((n, 3))
    return _normalize_rows(p)


def clustered_sphere_points(n, seed, n_clusters=4, width=0.05, frac=0.7):
    """A strongly non-uniform point set: `frac` of the points in Gaussian
    clusters of angular width `width` around random centres, the rest
    uniform.  Used to drive the tree to its depth limit."""
    rng = np.random.default_rng(seed)
    n_c = int(frac * n)
    centers = _normalize_rows(rng.standard_normal((n_clusters, 3)))
    which = rng.integers(0, n_clusters, n_c)
    p = centers[which] + width * rng.standard_normal((n_c, 3))
    u = rng.standard_normal((n - n_c, 3))
    return _normalize_rows(np.concatenate([p, u]))


def subset_indices(n, m, seed):
    """m distinct indices out of n, drawn without replacement, sorted."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(m, n), replace=False))
