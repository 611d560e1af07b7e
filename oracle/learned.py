"""O5b: the learned form's gated tree code, step by step.  TEST INFRASTRUCTURE ONLY.

The learned form replaces the fixed interpolation degree and the fixed
acceptance test by a decision per interaction:

* Candidates.  The traversal of Sec. 3 is run with a wider acceptance
  parameter theta_max.  A pair that is well separated at theta_max and has a
  side with more than N_T particles (a pair the method would approximate) is
  a candidate; pairs that are not separated are refined as usual, and pairs
  of two small nodes are PP as usual.
* Decision.  Each candidate is accepted at a degree class c (degree 4, 6, 8
  or 10) or rejected, from 12 features of the two nodes.
* Fallback.  A rejected candidate is traversed by the plain method from that
  pair on (parameter theta, the fallback degree), so with every candidate
  rejected the lists are those of the fixed-degree method.
* Evaluation.  PP as in Sec. 3; PC, CP and CC of an accepted candidate use
  the proxy points (source side) and interpolation points (target side) of
  that candidate's degree.

Features of a candidate (t, s), computed in FP64, rounded to float32 and then
to BF16 (R the chord between the circumcentres, r the circumradii, Q_x the
sum of |q| over node x, Q over all particles, w^(4) the source's degree-4
proxy charges):
  0 [n_t > N_T]        1 [n_s > N_T]        2 level_t / 8      3 level_s / 8
  4 r_t / R            5 r_s / R            6 (r_t + r_s) / R
  7 -log10 R / 2       8 log10(Q_s / Q) / 8 + 1                9 |sum_s q| / Q_s
 10 log10(|w^(4)|_1 / Q_s) / 2 (0 for a small source)         11 log10(Q_t / Q) / 8 + 1

Pair errors (labels): for candidate (t, s) and degree d, the largest over
t's particles of |approximation - exact| of the pair's contribution to W
(the sum before the cross product), the approximation being the one the pair
would get: PC (source proxies), CP (target interpolation) or CC (both).
"""

import numpy as np

from .geometry import node_level_key
from .interp import proxy_points, lagrange_matrix
from .mlp import bf16_round
from .tree import TreeCode, _pair_sum, well_separated

CLASS_DEGREES = (4, 6, 8, 10)


def _log10(v):
    return np.log10(max(v, 1e-30))


class LearnedTree(TreeCode):
    """TreeCode with per-interaction degree classes.  `decide` maps a
    (m, 16) array of BF16-rounded features to (accept (m,), class (m,));
    None rejects every candidate."""

    def __init__(self, x, zeta, area, theta=0.7, theta_max=None, degree=10, n_crit=64, max_level=None,
                 den="dist2", decide=None, kernel=None):
        super().__init__(x, zeta, area, theta=theta, degree=degree, n_crit=n_crit, max_level=max_level, den=den,
                         kernel=kernel)
        self.theta_max = theta if theta_max is None else theta_max
        self.fb_class = CLASS_DEGREES.index(degree)
        self._pcache = {}
        self._wcache = {}
        self.candidates = self._candidates()
        self.features = self.candidate_features(self.candidates)
        if decide is None or len(self.candidates) == 0:
            acc = np.zeros(len(self.candidates), dtype=bool)
            cls = np.zeros(len(self.candidates), dtype=np.int64)
        else:
            acc, cls = decide(self.features)
        self.accept, self.cls = np.asarray(acc, dtype=bool), np.asarray(cls, dtype=np.int64)
        self.lists, self.classes = self._gated_lists()

    # node data ----------------------------------------------------------------
    def level(self, node):
        return node_level_key(node)[0]

    def proxies_d(self, node, d):
        if (node, d) not in self._pcache:
            self._pcache[(node, d)] = proxy_points(self.geom.node_vertices(node), d)
        return self._pcache[(node, d)]

    def charges_d(self, node, d):
        """w_m = sum_j L_m(y_j) q_j at degree d (Sec. 3, particle-cluster)."""
        if (node, d) not in self._wcache:
            idx = self.ptree.members(node)
            L = lagrange_matrix(self.geom.node_vertices(node), d, self.x[idx])
            self._wcache[(node, d)] = L.T @ self.q[idx]
        return self._wcache[(node, d)]

    def qabs(self, node):
        return float(np.abs(self.q[self.ptree.members(node)]).sum())

    # traversal -------------------------------------------------------------------
    def _candidates(self):
        """Pairs separated at theta_max with a side of more than N_T particles,
        found by the traversal of Sec. 3 run at theta_max; sorted."""
        geom, cnt, NT = self.geom, self.ptree.count, self.n_crit
        out = []
        stack = [(t, s) for t in range(20) for s in range(20)]
        while stack:
            t, s = stack.pop()
            nt, ns = cnt[t], cnt[s]
            if nt == 0 or ns == 0:
                continue
            big_t, big_s = nt > NT, ns > NT
            if well_separated(geom, t, s, self.theta_max):
                if big_t or big_s:
                    out.append((t, s))
                continue
            if not big_t and not big_s:
                continue
            for pair in self._split(t, s):
                stack.append(pair)
        a = np.array(out, dtype=np.int64).reshape(-1, 2)
        return a[np.lexsort((a[:, 1], a[:, 0]))] if len(a) else a

    def _split(self, t, s):
        """Children pairs of a non-separated pair with a big side (Sec. 3
        refinement rule), or [] when neither side can be split."""
        cnt = self.ptree.count
        split_t = cnt[t] >= cnt[s]
        if split_t and not self.ptree.is_internal(t):
            split_t = False
        if not split_t and not self.ptree.is_internal(s):
            if self.ptree.is_internal(t):
                split_t = True
            else:
                return []
        if split_t:
            return [(c, s) for c in self.ptree.children(t) if cnt[c] > 0]
        return [(t, c) for c in self.ptree.children(s) if cnt[c] > 0]

    def _plain_from(self, t0, s0, lists, classes):
        """The plain traversal (theta, fallback class) from pair (t0, s0)."""
        geom, cnt, NT = self.geom, self.ptree.count, self.n_crit
        stack = [(t0, s0)]
        while stack:
            t, s = stack.pop()
            nt, ns = cnt[t], cnt[s]
            if nt == 0 or ns == 0:
                continue
            big_t, big_s = nt > NT, ns > NT
            if well_separated(geom, t, s, self.theta):
                kind = {(False, False): "PP", (False, True): "PC",
                        (True, False): "CP", (True, True): "CC"}[(big_t, big_s)]
                lists[kind].append((t, s))
                classes[kind].append(0 if kind == "PP" else self.fb_class)
                continue
            if not big_t and not big_s:
                lists["PP"].append((t, s))
                classes["PP"].append(0)
                continue
            kids = self._split(t, s)
            if not kids:
                lists["PP"].append((t, s))
                classes["PP"].append(0)
            stack.extend(kids)

    def _gated_lists(self):
        geom, cnt, NT = self.geom, self.ptree.count, self.n_crit
        lists = {"PP": [], "PC": [], "CP": [], "CC": []}
        classes = {"PP": [], "PC": [], "CP": [], "CC": []}
        # the part of the theta_max traversal that is not a candidate
        stack = [(t, s) for t in range(20) for s in range(20)]
        while stack:
            t, s = stack.pop()
            nt, ns = cnt[t], cnt[s]
            if nt == 0 or ns == 0:
                continue
            big_t, big_s = nt > NT, ns > NT
            if well_separated(geom, t, s, self.theta_max):
                if not big_t and not big_s:
                    lists["PP"].append((t, s))
                    classes["PP"].append(0)
                continue  # candidates are handled below
            if not big_t and not big_s:
                lists["PP"].append((t, s))
                classes["PP"].append(0)
                continue
            kids = self._split(t, s)
            if not kids:
                lists["PP"].append((t, s))
                classes["PP"].append(0)
            stack.extend(kids)
        for (t, s), acc, c in zip(self.candidates, self.accept, self.cls):
            t, s = int(t), int(s)
            if acc:
                kind = {(False, True): "PC", (True, False): "CP", (True, True): "CC"}[(cnt[t] > NT, cnt[s] > NT)]
                lists[kind].append((t, s))
                classes[kind].append(int(c))
            else:
                self._plain_from(t, s, lists, classes)
        out_l, out_c = {}, {}
        for k in lists:
            a = np.array(lists[k], dtype=np.int64).reshape(-1, 2)
            c = np.array(classes[k], dtype=np.int64)
            if len(a):
                o = np.lexsort((c, a[:, 1], a[:, 0]))
                a, c = a[o], c[o]
            out_l[k], out_c[k] = a, c
        return out_l, out_c

    # features -------------------------------------------------------------------
    def candidate_features(self, cands):
        geom, cnt = self.geom, self.ptree.count
        Q = sum(self.qabs(f) for f in range(20))
        F = np.zeros((len(cands), 16))
        for i, (t, s) in enumerate(cands):
            t, s = int(t), int(s)
            ct, cs = geom.node_center(t), geom.node_center(s)
            rt, rs = float(geom.node_radius(t)), float(geom.node_radius(s))
            dx = float(ct[0]) - float(cs[0])
            dy = float(ct[1]) - float(cs[1])
            dz = float(ct[2]) - float(cs[2])
            R = float(np.sqrt((dx * dx + dy * dy) + dz * dz))
            qs, qt = self.qabs(s), self.qabs(t)
            f = [float(cnt[t] > self.n_crit), float(cnt[s] > self.n_crit), self.level(t) / 8, self.level(s) / 8,
                 rt / R, rs / R, (rt + rs) / R, -_log10(R) / 2,
                 _log10(qs / Q if Q > 0 else 0.0) / 8 + 1,
                 abs(float(self.q[self.ptree.members(s)].sum())) / qs if qs > 0 else 0.0,
                 0.0, _log10(qt / Q if Q > 0 else 0.0) / 8 + 1]
            if cnt[s] > self.n_crit and qs > 0:
                f[10] = _log10(np.abs(self.charges_d(s, 4)).sum() / qs) / 2
            F[i, :12] = np.asarray(f, dtype=np.float64).astype(np.float32)
        return bf16_round(F)

    # evaluation --------------------------------------------------------------------
    def evaluate(self, parts=("near", "far")):
        x, q, k = self.x, self.q, self.kernel
        W = np.zeros((len(x), 3))
        what = set(parts)
        if "near" in what:
            for t, s in self.lists["PP"]:
                it, js = self.ptree.members(t), self.ptree.members(s)
                W[it] += _pair_sum(x[it], x[js], q[js], k, exclude_self=(t == s))
        if "far" in what:
            for (t, s), c in zip(self.lists["PC"], self.classes["PC"]):
                d = CLASS_DEGREES[c]
                it = self.ptree.members(t)
                W[it] += _pair_sum(x[it], self.proxies_d(s, d), self.charges_d(s, d), k)
            Wt = {}
            for name in ("CP", "CC"):
                for (t, s), c in zip(self.lists[name], self.classes[name]):
                    d = CLASS_DEGREES[c]
                    Wt.setdefault((t, d), np.zeros((len(self.proxies_d(t, d)), 3)))
                    if name == "CP":
                        js = self.ptree.members(s)
                        Wt[(t, d)] += _pair_sum(self.proxies_d(t, d), x[js], q[js], k)
                    else:
                        Wt[(t, d)] += _pair_sum(self.proxies_d(t, d), self.proxies_d(s, d), self.charges_d(s, d), k)
            for (t, d), vals in Wt.items():
                it = self.ptree.members(t)
                W[it] += lagrange_matrix(self.geom.node_vertices(t), d, x[it]) @ vals
        return W

    # labels ----------------------------------------------------------------------
    def pair_errors(self, cands=None):
        """(m, 4): for each candidate and degree class the largest error over
        the target's particles of the pair's approximate contribution to W."""
        cands = self.candidates if cands is None else cands
        x, q, k, cnt, NT = self.x, self.q, self.kernel, self.ptree.count, self.n_crit
        E = np.zeros((len(cands), 4))
        for i, (t, s) in enumerate(cands):
            t, s = int(t), int(s)
            it, js = self.ptree.members(t), self.ptree.members(s)
            exact = _pair_sum(x[it], x[js], q[js], k)
            for c, d in enumerate(CLASS_DEGREES):
                if cnt[t] <= NT:   # PC
                    ap = _pair_sum(x[it], self.proxies_d(s, d), self.charges_d(s, d), k)
                else:
                    if cnt[s] <= NT:   # CP
                        wt = _pair_sum(self.proxies_d(t, d), x[js], q[js], k)
                    else:              # CC
                        wt = _pair_sum(self.proxies_d(t, d), self.proxies_d(s, d), self.charges_d(s, d), k)
                    ap = lagrange_matrix(self.geom.node_vertices(t), d, x[it]) @ wt
                E[i, c] = np.sqrt(((ap - exact) ** 2).sum(1)).max()
        return E


def labels_from_errors(E, tol):
    """accept iff some class meets tol; ordinal targets: smallest such class
    above class k (k = 0, 1, 2)."""
    E = np.asarray(E)
    ok = E <= tol
    cmin = np.where(ok.any(1), ok.argmax(1), 4)
    y = np.zeros((len(E), 4), dtype=np.float32)
    y[:, 0] = cmin < 4
    for k in range(3):
        y[:, k + 1] = (cmin < 4) & (cmin > k)
    return y
