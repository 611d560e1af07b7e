"""O6: adaptive mesh refinement of the particle triangulation (Appendix A;
Gaussian-vortex test of Sec. 4.3).  TEST INFRASTRUCTURE ONLY.

The particles are the vertices of a triangulation of the sphere with a tree
structure: every triangle of the initial mesh (the icosahedral grid's faces)
is the root of a refinement tree; its leaves are the current triangles.  One
adaptation pass, run after every time step, tests each triangle T with
vertices a, b, c (current positions and vorticities):

    C(T):  |A_T (zeta_a + zeta_b + zeta_c) / 3| >= eps1   (circulation)
        or max(zeta) - min(zeta)               >= eps2   (variation)

A_T the area of T (see the quadrature reading below).  A leaf with C(T) at
depth below max_levels is split into four, (a, m_ab, m_ca), (m_ab, b, m_bc),
(m_ca, m_bc, c), (m_ab, m_bc, m_ca); a refined triangle whose four children
are leaves and for which C(T) no longer holds is merged back (never below the
initial mesh).

Readings where the appendix is silent (the same in the GPU library):

* The test of the circulation uses its magnitude (a strong vortex of either
  sign is refined).
* All decisions of a pass use the positions and vorticities at the start of
  the pass; merging is decided before splitting (a triangle merged in a pass
  is not split in it), so a pass changes the depth of any region by at most
  one level.
* A midpoint particle is shared by the two triangles of its edge: it is
  created by whichever side splits first and removed when no leaf triangle
  has it as a vertex.  Its position is (x_a + x_b) / |x_a + x_b| of the edge
  ends' current positions.
* Its vorticity: the absolute vorticity zeta + 2 Omega z is carried
  unchanged by every particle (dzeta/dt = -2 Omega dz/dt), so the new
  particle takes the mean absolute vorticity of the edge ends minus
  2 Omega z at its own position.
* Areas are Lagrangian (the flow is incompressible, and without refinement
  the paper keeps every A_i constant in time): each triangle carries the
  area it was given when created -- an initial triangle its spherical area
  (Van Oosterom-Strackee) at the start, the four children of a split the
  parent's carried area in proportion to their spherical areas at the
  moment of the split -- and a merged triangle gets back its own carried
  area (the sum of its children's).  The straight-edged triangle of a
  distorted mesh no longer bounds the material patch, so areas recomputed
  from current positions grow without bound where the flow folds the mesh.
  Quadrature weights: A_i = sum over the leaf triangles having i as a
  vertex of A_T / 3 (the barycentric-dual areas of the initial grid); they
  sum to 4 pi at every pass.
* Each call of ``adapt`` is one pass; an initial condition given as a
  function is resolved by alternating passes with re-evaluating the
  function at the particles (``resolve_initial``).

Operation order of every floating-point expression is the one written in
the code, so another implementation of the same recipe takes the same
decisions.
"""

import numpy as np

LEAF, REFINED = 1, 2


def tri_area(a, b, c):
    """Spherical area of the triangle (a, b, c), unit vectors
    (Van Oosterom-Strackee): 2 atan2(|a . (b x c)|, 1 + a.b + b.c + c.a)."""
    bxc0 = b[1] * c[2] - b[2] * c[1]
    bxc1 = b[2] * c[0] - b[0] * c[2]
    bxc2 = b[0] * c[1] - b[1] * c[0]
    trip = abs((a[0] * bxc0 + a[1] * bxc1) + a[2] * bxc2)
    ab = (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]
    bc = (b[0] * c[0] + b[1] * c[1]) + b[2] * c[2]
    ca = (c[0] * a[0] + c[1] * a[1]) + c[2] * a[2]
    return 2.0 * float(np.arctan2(trip, ((1.0 + ab) + bc) + ca))


def criterion(area, za, zb, zc, eps1, eps2):
    """C(T) for a triangle of area `area` with vertex vorticities za, zb, zc."""
    circ = area * (((za + zb) + zc) / 3.0)
    spread = max(za, zb, zc) - min(za, zb, zc)
    return abs(circ) >= eps1 or spread >= eps2


def midpoint(xa, xb):
    s0, s1, s2 = xa[0] + xb[0], xa[1] + xb[1], xa[2] + xb[2]
    r = np.sqrt((s0 * s0 + s1 * s1) + s2 * s2)
    return np.array([s0 / r, s1 / r, s2 / r])


class Mesh:
    """The adaptive particle triangulation.  x0 (n0, 3), zeta0 (n0,) the
    initial particles, faces (F, 3) the initial triangles over them."""

    def __init__(self, x0, zeta0, faces, eps1, eps2, omega, max_levels=3):
        self.eps1, self.eps2, self.omega, self.max_levels = float(eps1), float(eps2), float(omega), int(max_levels)
        self.x = [np.array(p, dtype=np.float64) for p in np.asarray(x0, dtype=np.float64)]
        self.zeta = [float(v) for v in np.asarray(zeta0, dtype=np.float64)]
        self.alive = [True] * len(self.x)
        self.edge_mid = {}          # (min, max) particle pair -> midpoint particle
        # triangles: vertices, depth, state, children (list of 4 ids or None), carried area
        self.tv, self.depth, self.state, self.children, self.tarea = [], [], [], [], []
        self.roots = []
        for f in np.asarray(faces, dtype=np.int64):
            i, j, k = (int(v) for v in f)
            t = self._new_tri((i, j, k), 0)
            self.tarea[t] = tri_area(self.x[i], self.x[j], self.x[k])
            self.roots.append(t)

    def _new_tri(self, v, depth):
        self.tv.append(v)
        self.depth.append(depth)
        self.state.append(LEAF)
        self.children.append(None)
        self.tarea.append(0.0)
        return len(self.tv) - 1

    # -- the particle state -------------------------------------------------------
    def particles(self):
        """(ids, x (n, 3), zeta (n,), area (n,)) of the live particles, in
        increasing particle id."""
        ids = [i for i, a in enumerate(self.alive) if a]
        area = self.areas()
        return (np.array(ids, dtype=np.int64), np.array([self.x[i] for i in ids]).reshape(-1, 3),
                np.array([self.zeta[i] for i in ids]), np.array([area[i] for i in ids]))

    def set_state(self, ids, x, zeta):
        for k, i in enumerate(ids):
            self.x[i] = np.array(x[k], dtype=np.float64)
            self.zeta[i] = float(zeta[k])

    def leaves(self):
        return [t for t in range(len(self.tv)) if self.state[t] == LEAF]

    def areas(self):
        a = [0.0] * len(self.x)
        for t in self.leaves():
            i, j, k = self.tv[t]
            w = self.tarea[t] / 3.0
            a[i] += w
            a[j] += w
            a[k] += w
        return a

    # -- one adaptation pass -----------------------------------------------------------
    def _crit(self, t):
        i, j, k = self.tv[t]
        return criterion(self.tarea[t], self.zeta[i], self.zeta[j], self.zeta[k], self.eps1, self.eps2)

    def _mid(self, a, b):
        key = (min(a, b), max(a, b))
        m = self.edge_mid.get(key)
        if m is not None and self.alive[m]:
            return m
        xm = midpoint(self.x[a], self.x[b])
        two_om = 2.0 * self.omega
        absv = 0.5 * ((self.zeta[a] + two_om * self.x[a][2]) + (self.zeta[b] + two_om * self.x[b][2]))
        zm = absv - two_om * xm[2]
        if m is None:
            self.x.append(xm)
            self.zeta.append(zm)
            self.alive.append(True)
            m = len(self.x) - 1
            self.edge_mid[key] = m
        else:                      # the edge had a midpoint earlier: the particle comes back
            self.x[m], self.zeta[m], self.alive[m] = xm, zm, True
        return m

    def adapt(self):
        """One pass; returns (merged, split) triangle counts."""
        ntri = len(self.tv)
        crit = {}
        for t in range(ntri):
            if self.state[t] == LEAF or (self.state[t] == REFINED and
                                         all(self.state[c] == LEAF for c in self.children[t])):
                crit[t] = self._crit(t)
        merged = [t for t in range(ntri) if self.state[t] == REFINED
                  and all(self.state[c] == LEAF for c in self.children[t]) and not crit[t]]
        gone = set()
        for t in merged:
            for c in self.children[t]:
                self.state[c] = 0
                gone.add(c)
            self.state[t] = LEAF
        split = [t for t in range(ntri) if self.state[t] == LEAF and t not in merged and t not in gone
                 and crit[t] and self.depth[t] < self.max_levels]
        for t in split:
            a, b, c = self.tv[t]
            mab, mbc, mca = self._mid(a, b), self._mid(b, c), self._mid(c, a)
            if self.children[t] is None:
                d = self.depth[t] + 1
                self.children[t] = [self._new_tri((a, mab, mca), d), self._new_tri((mab, b, mbc), d),
                                    self._new_tri((mca, mbc, c), d), self._new_tri((mab, mbc, mca), d)]
            else:
                for ch in self.children[t]:
                    self.state[ch] = LEAF
            # the parent's carried area, shared in proportion to the children's spherical areas
            g = [tri_area(*(self.x[v] for v in self.tv[ch])) for ch in self.children[t]]
            gs = ((g[0] + g[1]) + g[2]) + g[3]
            for ch, gc in zip(self.children[t], g):
                self.tarea[ch] = self.tarea[t] * (gc / gs)
            self.state[t] = REFINED
        used = set()
        for t in self.leaves():
            used.update(self.tv[t])
        for i in range(len(self.alive)):
            self.alive[i] = i in used
        return len(merged), len(split)

    def resolve_initial(self, zeta_fn, passes=None):
        """Alternate passes with zeta = zeta_fn(x) at every live particle until
        a pass changes nothing (at most max_levels + 1 passes)."""
        passes = self.max_levels + 1 if passes is None else passes
        for _ in range(passes):
            ids, x, _, _ = self.particles()
            z = zeta_fn(x)
            for k, i in enumerate(ids):
                self.zeta[i] = float(z[k])
            m, s = self.adapt()
            ids, x, _, _ = self.particles()
            z = zeta_fn(x)
            for k, i in enumerate(ids):
                self.zeta[i] = float(z[k])
            if m == 0 and s == 0:
                break


def step_with_amr(mesh, dt, velocity_fn, rk4_step):
    """One RK4 step of the live particles (velocity_fn(x, zeta, area)), then
    one adaptation pass."""
    ids, x, z, a = mesh.particles()
    xn, zn = rk4_step(x, z, a, dt, mesh.omega, velocity_fn)
    mesh.set_state(ids, xn, zn)
    return mesh.adapt()
