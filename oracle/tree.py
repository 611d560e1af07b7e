"""O2: the spherical tree code, step by step.  TEST INFRASTRUCTURE ONLY.

Follows Sec. 3 of the paper (treatment of clusters; dual tree traversal) with
these readings where it is silent or written for a scalar kernel:

* Vector kernel.  The velocity is u_i = -(1/4pi) x_i x W_i with
  W_i = sum_j q_j K(x_i, y_j), K(x, y) = (y - x) / den(x, y), q_j = zeta_j A_j.
  Because x_i x x_i = 0 this is exactly the paper's sum (Sec. 2, discrete
  system); the cross product is taken once, after all interactions, so
  x_i . u_i = 0 holds for every approximation.
* Source side (PC, CC): K(x, .) is interpolated in the source triangle with
  scalar charges: proxy charges w_m = sum_j L_m(y_j) q_j, which equals
  V^{-T} omega with the paper's proxy weights omega_k = sum_j B_k(y_j) q_j.
* Target side (CP, CC): the function x -> sum_j q_j K(x, y_j) (three
  components, K as above) is interpolated in the target triangle from its
  values at the target's interpolation points.  Interpolating this form
  rather than sum_j q_j y_j / den keeps the interpolated quantity of the
  size of the velocity, so the later cross product cancels nothing.
* "Many particles" means count > N_T.  A node is internal iff count > N_T and
  level < max_level.
* Well separated iff (r_t + r_s) / R < theta, evaluated as
  s * s < (theta * theta) * R2 with s = r_t + r_s and
  R2 = (dx*dx + dy*dy) + dz*dz, dx = c_t - c_s componentwise.
* Traversal from the 20 x 20 root pairs: empty nodes are skipped; if well
  separated, the pair is PP / PC / CP / CC by which side has many particles;
  otherwise, if neither has many particles, PP; otherwise the side with more
  particles is split (tie: the target); if it is not internal the other side
  is split; if neither is internal the pair is PP.
"""

import numpy as np

from .geometry import TreeGeometry, ParticleTree, node_level_key, level_offset
from .interp import proxy_points, lagrange_matrix, n_basis

FOUR_PI = 4.0 * np.pi


def default_max_level(n, n_crit):
    """Depth limit: two levels below the level where an average node of a
    uniform distribution holds N_T particles, capped at 12."""
    lvl = 0
    while 20 * 4 ** lvl * n_crit < n:
        lvl += 1
    return min(12, lvl + 2)


# --- kernels -----------------------------------------------------------------

def biot_savart_kernel(den="dot"):
    """K(X, Y) = (Y - X) / den(X, Y) for X (a, 3), Y (b, 3) -> (a, b, 3)."""
    def k(X, Y):
        D = Y[None, :, :] - X[:, None, :]
        if den == "dot":
            dn = 1.0 - ((X[:, None, 0] * Y[None, :, 0] + X[:, None, 1] * Y[None, :, 1])
                        + X[:, None, 2] * Y[None, :, 2])
        else:
            dn = 0.5 * ((D[..., 0] * D[..., 0] + D[..., 1] * D[..., 1]) + D[..., 2] * D[..., 2])
        return D / dn[..., None]
    return k


def stream_kernel(den="dot"):
    """The stream function's kernel log(den(X, Y)) in component 0 (the other
    two components zero), so that the same interactions carry it; the
    stream function is psi = W_0 / 4 pi (Sec. 2, stream function)."""
    def k(X, Y):
        if den == "dot":
            dn = 1.0 - ((X[:, None, 0] * Y[None, :, 0] + X[:, None, 1] * Y[None, :, 1])
                        + X[:, None, 2] * Y[None, :, 2])
        else:
            D = Y[None, :, :] - X[:, None, :]
            dn = 0.5 * ((D[..., 0] * D[..., 0] + D[..., 1] * D[..., 1]) + D[..., 2] * D[..., 2])
        out = np.zeros(dn.shape + (3,))
        out[..., 0] = np.log(dn)
        return out
    return k


def polynomial_kernel(d, a=(0.3, -0.5, 0.7)):
    """A test kernel homogeneous of degree d in both arguments:
    K(x, y) = a (x . y)^d.  Interpolation of degree d reproduces it exactly."""
    a = np.asarray(a, dtype=np.float64)

    def k(X, Y):
        dot = X @ Y.T
        return (dot ** d)[..., None] * a[None, None, :]
    return k


def _pair_sum(xt, xs, q, kernel, exclude_self=False):
    with np.errstate(divide="ignore", invalid="ignore"):
        K = kernel(xt, xs)
    if exclude_self:
        # the j = i term is excluded (Sec. 2, discrete system: j != i)
        ii = np.arange(len(xt))
        K[ii, ii, :] = 0.0
    return (q[None, :, None] * K).sum(1)


# --- traversal -----------------------------------------------------------------

def well_separated(geom, t, s, theta):
    ct, cs = geom.node_center(t), geom.node_center(s)
    rt, rs = geom.node_radius(t), geom.node_radius(s)
    dx = float(ct[0]) - float(cs[0])
    dy = float(ct[1]) - float(cs[1])
    dz = float(ct[2]) - float(cs[2])
    R2 = (dx * dx + dy * dy) + dz * dz
    s_ = rt + rs
    return s_ * s_ < (theta * theta) * R2


def traverse(ptree, theta):
    """Dual tree traversal -> dict of lists PP, PC, CP, CC of (t, s) node ids,
    each sorted by (t, s)."""
    geom = ptree.geom
    NT = ptree.n_crit
    cnt = ptree.count
    lists = {"PP": [], "PC": [], "CP": [], "CC": []}
    stack = [(t, s) for t in range(20) for s in range(20)]
    stack.reverse()
    while stack:
        t, s = stack.pop()
        nt, ns = cnt[t], cnt[s]
        if nt == 0 or ns == 0:
            continue
        big_t, big_s = nt > NT, ns > NT
        if well_separated(geom, t, s, theta):
            kind = {(False, False): "PP", (False, True): "PC",
                    (True, False): "CP", (True, True): "CC"}[(big_t, big_s)]
            lists[kind].append((t, s))
            continue
        if not big_t and not big_s:
            lists["PP"].append((t, s))
            continue
        split_t = nt >= ns
        if split_t and not ptree.is_internal(t):
            split_t = False
        if not split_t and not ptree.is_internal(s):
            if ptree.is_internal(t):
                split_t = True
            else:
                lists["PP"].append((t, s))
                continue
        if split_t:
            for c in ptree.children(t):
                if cnt[c] > 0:
                    stack.append((c, s))
        else:
            for c in ptree.children(s):
                if cnt[c] > 0:
                    stack.append((t, c))
    out = {}
    for k, v in lists.items():
        a = np.array(v, dtype=np.int64).reshape(-1, 2)
        if len(a):
            a = a[np.lexsort((a[:, 1], a[:, 0]))]
        out[k] = a
    return out


# --- the tree code ---------------------------------------------------------------

class TreeCode:
    """One velocity evaluation of the spherical tree code."""

    def __init__(self, x, zeta, area, theta=0.7, degree=8, n_crit=64,
                 max_level=None, den="dot", kernel=None):
        self.x = np.asarray(x, dtype=np.float64)
        self.q = np.asarray(zeta, dtype=np.float64) * np.asarray(area, dtype=np.float64)
        n = len(self.x)
        self.theta, self.degree, self.n_crit = theta, degree, n_crit
        self.max_level = default_max_level(n, n_crit) if max_level is None else max_level
        self.kernel = biot_savart_kernel(den) if kernel is None else kernel
        self.geom = TreeGeometry(self.max_level)
        self.ptree = ParticleTree(self.x, self.geom, n_crit)
        self.lists = traverse(self.ptree, theta)
        self._proxy_cache = {}

    # proxies and proxy charges ---------------------------------------------------
    def proxies(self, node):
        if node not in self._proxy_cache:
            self._proxy_cache[node] = proxy_points(self.geom.node_vertices(node), self.degree)
        return self._proxy_cache[node]

    def proxy_charges(self, node):
        """w_m = sum_{j in node} L_m(y_j) q_j (Sec. 3, particle-cluster)."""
        idx = self.ptree.members(node)
        L = lagrange_matrix(self.geom.node_vertices(node), self.degree, self.x[idx])
        return L.T @ self.q[idx]

    def all_proxy_charges(self):
        big = np.nonzero(self.ptree.count > self.n_crit)[0]
        return {int(b): self.proxy_charges(int(b)) for b in big}

    # interactions ----------------------------------------------------------------
    def evaluate(self, parts=("near", "far")):
        """Returns W (N, 3) in input order (the sum before the cross product)."""
        x, q, k = self.x, self.q, self.kernel
        n = len(x)
        W = np.zeros((n, 3))
        what = set(parts)
        wq = self.all_proxy_charges() if (self.lists["PC"].size or self.lists["CC"].size) else {}
        if "near" in what:
            for t, s in self.lists["PP"]:
                it, js = self.ptree.members(t), self.ptree.members(s)
                W[it] += _pair_sum(x[it], x[js], q[js], k, exclude_self=(t == s))
        if "far" in what:
            for t, s in self.lists["PC"]:
                it = self.ptree.members(t)
                W[it] += _pair_sum(x[it], self.proxies(s), wq[s], k)
            Wt = {}
            for t, s in self.lists["CP"]:
                js = self.ptree.members(s)
                Wt.setdefault(t, np.zeros((n_basis(self.degree), 3)))
                Wt[t] += _pair_sum(self.proxies(t), x[js], q[js], k)
            for t, s in self.lists["CC"]:
                Wt.setdefault(t, np.zeros((n_basis(self.degree), 3)))
                Wt[t] += _pair_sum(self.proxies(t), self.proxies(s), wq[s], k)
            self.target_values = Wt
            # target side: interpolate W from the target's points to its particles
            for t, vals in Wt.items():
                it = self.ptree.members(t)
                L = lagrange_matrix(self.geom.node_vertices(t), self.degree, x[it])
                W[it] += L @ vals
        return W

    def velocity(self, parts=("near", "far")):
        W = self.evaluate(parts)
        return -np.cross(self.x, W) / FOUR_PI

    def stream_function(self, parts=("near", "far")):
        """psi_i = W_0 / 4 pi for a TreeCode built with kernel=stream_kernel()."""
        return self.evaluate(parts)[:, 0] / FOUR_PI

    def list_counts(self):
        return {k: len(v) for k, v in self.lists.items()}

    def kernel_evaluations(self):
        """Number of kernel evaluations the lists imply (PP self pairs count
        n_t (n_t - 1))."""
        c = self.ptree.count
        npx = n_basis(self.degree)
        tot = 0
        for t, s in self.lists["PP"]:
            tot += c[t] * c[s] - (c[t] if t == s else 0)
        tot += sum(c[t] * npx for t, _ in self.lists["PC"])
        tot += sum(npx * c[s] for _, s in self.lists["CP"])
        tot += npx * npx * len(self.lists["CC"])
        return int(tot)


def velocity(x, zeta, area, **kw):
    return TreeCode(x, zeta, area, **kw).velocity()


__all__ = ["TreeCode", "velocity", "traverse", "well_separated", "default_max_level",
           "biot_savart_kernel", "stream_kernel", "polynomial_kernel", "node_level_key", "level_offset"]
