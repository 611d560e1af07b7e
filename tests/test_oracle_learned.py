"""Pins of the learned form's oracle (CPU): the network's gradient against
finite differences and closed forms, BF16 rounding, the gated traversal's
coverage under any decisions, and the pair errors against cases whose answer
is known."""

import numpy as np
import pytest

import synthetic as S
from oracle import mlp
from oracle import learned as OL
from oracle import tree as otree
from oracle.tree import polynomial_kernel


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((n, 16))
    x[:, :12] = rng.uniform(-1, 1, (n, 12))
    y = (rng.uniform(size=(n, 4)) < 0.5).astype(np.float64)
    return x, y


def test_gradient_matches_finite_differences():
    x, y = _data(37, 1)
    th = mlp.init_params(3) + 0.05 * np.random.default_rng(4).standard_normal(mlp.N_PARAMS)
    g = mlp.grad(th, x, y)
    rng = np.random.default_rng(5)
    idx = np.concatenate([rng.choice(np.arange(o, o + int(np.prod(sh))), 12, replace=False)
                          for o, sh in mlp.SLICES.values() if np.prod(sh) > 12] + [np.arange(5248, 5252)])
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss(th + e, x, y) - mlp.loss(th - e, x, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, np.abs(g).max()), i


def test_loss_and_output_bias_gradient_closed_form():
    # all weights zero: outputs = b3 for every row
    b3 = np.array([0.3, -1.2, 0.7, 2.0])
    th = mlp.pack({"W1": np.zeros((12, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
                   "W3": np.zeros((64, 4)), "b3": b3})
    x, y = _data(10, 2)
    sig = 1 / (1 + np.exp(-b3))
    soft = np.log1p(np.exp(b3))            # BCE(o, y) = log(1 + e^o) - o y
    wr, wh = mlp.W_REJECT, mlp.W_HIGHER

    def row(r):                            # reject rows weigh wr, "higher degree" targets wh
        a = wr if r[0] == 0 else 1.0
        return a * (soft[0] - b3[0] * r[0]) + r[0] * sum((wh if r[k] == 1 else 1.0) * (soft[k] - b3[k] * r[k])
                                                          for k in (1, 2, 3))
    want = np.mean([row(r) for r in y])
    assert abs(mlp.loss(th, x, y) - want) < 1e-14
    g = mlp.unpack(mlp.grad(th, x, y))["b3"]
    assert abs(g[0] - np.mean(np.where(y[:, 0] == 0, wr, 1.0) * (sig[0] - y[:, 0]))) < 1e-14
    for k in (1, 2, 3):
        assert abs(g[k] - np.mean(y[:, 0] * np.where(y[:, k] == 1, wh, 1.0) * (sig[k] - y[:, k]))) < 1e-14


def test_weighted_optimum_of_a_constant_network():
    # all weights zero: the loss is minimised over b3 where its gradient
    # vanishes, at the labels' log-odds with the reject rows (acceptance) and
    # the "higher degree" targets among accepted rows (ordinals) counted
    # W_REJECT and W_HIGHER times: o0 = ln(n1 / (W_REJECT n0)),
    # ok = ln(W_HIGHER m1 / m0)
    x, y = _data(60, 7)
    n1, n0 = y[:, 0].sum(), (1 - y[:, 0]).sum()
    acc = y[:, 0] == 1
    b3 = np.empty(4)
    b3[0] = np.log(n1 / (mlp.W_REJECT * n0))
    for k in (1, 2, 3):
        m1, m0 = y[acc, k].sum(), (1 - y[acc, k]).sum()
        b3[k] = np.log(mlp.W_HIGHER * m1 / m0)
    th = mlp.pack({"W1": np.zeros((12, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
                   "W3": np.zeros((64, 4)), "b3": b3})
    g = mlp.unpack(mlp.grad(th, x, y))["b3"]
    assert np.abs(g).max() < 1e-14
    # the unweighted log-odds are not the optimum: the weights move it by ln W
    b3[0] += np.log(mlp.W_REJECT)
    th2 = mlp.pack({"W1": np.zeros((12, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
                    "W3": np.zeros((64, 4)), "b3": b3})
    assert mlp.unpack(mlp.grad(th2, x, y))["b3"][0] > 1e-3


def test_bf16_rounding_ties_to_even():
    vals = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -2.5, 1 + 2 ** -9])
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, 1.0])
    assert np.array_equal(mlp.bf16_round(vals), want)
    assert np.array_equal(mlp.from_bf16_bits(mlp.bf16_bits(vals)), want)


def _coverage(lt, n):
    c = np.zeros((n, n), dtype=np.int64)
    for name in ("PP", "PC", "CP", "CC"):
        for t, s in lt.lists[name]:
            it, js = lt.ptree.members(t), lt.ptree.members(s)
            c[np.ix_(it, js)] += 1
    return c


def _case(level=3, seed=7):
    x = S.icosahedral_grid(level) @ S.random_rotation(seed).T
    z = S.rossby_haurwitz(x, 4) + S.gaussian_vortex(x, seed=seed, amplitude=1e-4)
    return x, z, S.uniform_areas(len(x))


def test_reject_all_is_the_fixed_degree_method():
    x, z, a = _case()
    lt = OL.LearnedTree(x, z, a, theta=0.6, theta_max=0.8, degree=10, n_crit=16)
    ref = otree.TreeCode(x, z, a, theta=0.6, degree=10, n_crit=16, den="dist2")
    assert len(lt.candidates) > 0
    for k in ("PP", "PC", "CP", "CC"):
        assert np.array_equal(lt.lists[k], ref.lists[k]), k
        assert (lt.classes[k][lt.classes[k] > -1] == (0 if k == "PP" else 3)).all()
    assert np.abs(lt.velocity() - ref.velocity()).max() <= 1e-13 * np.abs(ref.velocity()).max()


@pytest.mark.parametrize("rule", ["accept_all", "random"])
def test_any_decisions_cover_every_pair_once(rule):
    x, z, a = _case()
    rng = np.random.default_rng(11)

    def decide(F):
        m = len(F)
        if rule == "accept_all":
            return np.ones(m, bool), np.full(m, 2)
        return rng.uniform(size=m) < 0.6, rng.integers(0, 4, m)

    lt = OL.LearnedTree(x, z, a, theta=0.6, theta_max=0.9, degree=8, n_crit=16, decide=decide)
    n = len(x)
    c = _coverage(lt, n)
    np.testing.assert_array_equal(c, np.ones((n, n), dtype=np.int64))
    # and the result is a tree-code approximation of the direct sum
    from oracle import direct
    ud = direct.velocity(x, z, a, den="dist2")
    e = np.sqrt(((lt.velocity() - ud) ** 2).sum() / (ud ** 2).sum())
    assert e < 1e-2


def test_pair_errors_vanish_for_a_kernel_in_the_interpolation_space():
    # K(x, y) = a (x . y)^4 lies in the degree-4 space in both arguments, so
    # every class (degree >= 4) reproduces it: PC, CP and CC alike
    x, z, a = _case(level=3, seed=5)
    lt = OL.LearnedTree(x, z, a, theta=0.6, theta_max=0.9, degree=10, n_crit=16, kernel=polynomial_kernel(4))
    E = lt.pair_errors()
    cnt = lt.ptree.count
    kinds = {(cnt[t] > 16, cnt[s] > 16) for t, s in lt.candidates}
    assert {(False, True), (True, False), (True, True)} <= kinds
    scale = np.abs(lt.q).sum()
    assert E.max() < 1e-11 * scale
    # degree 5 is outside the degree-4 class: the negative control must fail
    lt5 = OL.LearnedTree(x, z, a, theta=0.6, theta_max=0.9, degree=10, n_crit=16, kernel=polynomial_kernel(5))
    assert lt5.pair_errors()[:, 0].max() > 1e-6 * scale


def test_pair_errors_fall_with_degree():
    x, z, a = _case(level=4, seed=3)
    lt = OL.LearnedTree(x, z, a, theta=0.6, theta_max=0.8, degree=10, n_crit=32)
    E = lt.pair_errors()
    med = np.median(E, axis=0)
    assert med[0] > med[1] > med[2] > med[3]
    # and the candidates' features sit inside the acceptance region (f6 =
    # (r_t + r_s)/R < theta_max up to BF16 rounding)
    F = lt.features
    assert (F[:, 6] <= 0.8 * (1 + 2 ** -8)).all()
    assert ((F[:, 9] >= 0) & (F[:, 9] <= 1)).all()
    np.testing.assert_allclose(F[:, 4] + F[:, 5], F[:, 6], rtol=2 ** -7)


def test_labels_from_errors():
    E = np.array([[1e-9, 1e-10, 1e-11, 1e-12],
                  [1e-5, 1e-7, 1e-9, 1e-12],
                  [1e-5, 1e-6, 1e-7, 1e-8],
                  [1e-5, 1e-9, 1e-6, 1e-6]])
    y = OL.labels_from_errors(E, 1e-8)
    np.testing.assert_array_equal(y, [[1, 0, 0, 0], [1, 1, 1, 0], [1, 1, 1, 1], [1, 1, 0, 0]])
    y = OL.labels_from_errors(E, 1e-13)
    np.testing.assert_array_equal(y[:, 0], [0, 0, 0, 0])


def test_features_of_one_candidate_by_hand():
    """The twelve features of one candidate worked out by hand.  Faces 0 and
    19 are antipodal root triangles (circumcentres c and -c, so R = 2; the
    circumradius r0 follows from the icosahedron, cos(angle) = phi^2 /
    (sqrt 3 sqrt(1 + phi^2))).  N_T = 1, depth limit 0, theta_max = 0.9, so
    the candidates are (0, 19) and (19, 0).  Target face 0 holds charges 1
    and -0.5; source face 19 holds charges 2 and -1 placed exactly on two of
    its interior degree-4 interpolation points (barycentrics written out from
    the Gauss-Lobatto nodes 1/2 -+ sqrt(3/7)/2 and 1/2), where the degree-4
    proxy charges are the charges themselves (L_m(y_j) = delta), so
    |w^(4)|_1 = Q_s."""
    from oracle import geometry as G
    geom = G.TreeGeometry(0)
    va, vb = geom.node_vertices(0), geom.node_vertices(19)
    assert np.abs(geom.node_center(0) + geom.node_center(19)).max() < 1e-15
    r = np.sqrt(3.0 / 7.0) / 2.0
    bary = [((1 - r) / 3, (1 - r) / 3, (1 + 2 * r) / 3),     # point (1, 1, 2)
            ((1 + 2 * r) / 3, (1 - r) / 3, (1 - r) / 3)]     # point (2, 1, 1)
    src = []
    for b in bary:
        p = b[0] * vb[0] + b[1] * vb[1] + b[2] * vb[2]
        src.append(p / np.linalg.norm(p))
    ca = (va[0] + va[1] + va[2]) / 3.0
    tgt = [ca / np.linalg.norm(ca), (0.8 * ca + 0.2 * va[0]) / np.linalg.norm(0.8 * ca + 0.2 * va[0])]
    x = np.array(tgt + src)
    q = np.array([1.0, -0.5, 2.0, -1.0])
    lt = OL.LearnedTree(x, q, np.ones(4), theta=0.6, theta_max=0.9, degree=4, n_crit=1, max_level=0)
    assert lt.candidates.tolist() == [[0, 19], [19, 0]]
    phi = (1 + 5 ** 0.5) / 2
    cos_a = phi ** 2 / (3 ** 0.5 * (1 + phi ** 2) ** 0.5)
    r0 = (2 - 2 * cos_a) ** 0.5
    Q, Qs, Qt = 4.5, 3.0, 1.5
    want = [1, 1, 0, 0, r0 / 2, r0 / 2, r0, -np.log10(2.0) / 2, np.log10(Qs / Q) / 8 + 1, 1.0 / 3.0, 0.0,
            np.log10(Qt / Q) / 8 + 1]
    got = lt.features[0, :12]
    for k in range(12):
        # BF16 keeps 8 significant bits: one unit in the last place
        assert abs(got[k] - want[k]) <= 2.0 ** -8 * max(abs(want[k]), 1e-6), (k, got[k], want[k])
    assert np.all(lt.features[:, 12:] == 0)
    # the reverse pair swaps the node roles (its f10 depends on where the
    # target's charges sit, so it is not checked)
    back = lt.features[1, :12]
    want_b = [1, 1, 0, 0, r0 / 2, r0 / 2, r0, -np.log10(2.0) / 2, np.log10(Qt / Q) / 8 + 1, 1.0 / 3.0, None,
              np.log10(Qs / Q) / 8 + 1]
    for k in range(12):
        if want_b[k] is not None:
            assert abs(back[k] - want_b[k]) <= 2.0 ** -8 * max(abs(want_b[k]), 1e-6), (k, back[k], want_b[k])


def test_calibration_shifts_hand_case():
    """Bias calibration on ten hand-made samples.  Rejected labels with
    acceptance logits 0.5, 2.0, -1.0 and max_false_accept 0.1: at most one of
    ten may stay accepted, so the shift must reach 0.5 (o0 - d > 0 is strict)
    -- the first grid value at or above 0.5 is 1e-3 * 64000^(112/199).  Of
    the seven accepted samples (o0 = 3) one needs two ordinal steps with
    logits (1.0, -0.3, -2.0): it is under-classed until -0.3 + d > 0, and 1/7
    exceeds max_under_class 0.1, so dc is the first grid value above 0.3,
    1e-3 * 64000^(103/199)."""
    from oracle import mlp
    out = np.zeros((10, 4))
    y = np.zeros((10, 4))
    out[:3, 0] = [0.5, 2.0, -1.0]
    out[3:, 0] = 3.0
    out[3:, 1:] = -5.0
    y[3:, 0] = 1.0
    out[4, 1:] = [1.0, -0.3, -2.0]
    y[4, 1:] = [1.0, 1.0, 0.0]
    grid = mlp.calibration_grid()
    assert grid[112] < 0.5 < grid[113] and grid[103] < 0.3 < grid[104]
    da, dc = mlp.calibration_shifts(out, y, 0.1, 0.1)
    assert da == pytest.approx(1e-3 * 64000.0 ** (112 / 199), rel=1e-14)
    assert dc == pytest.approx(1e-3 * 64000.0 ** (103 / 199), rel=1e-14)
    # looser bars: every false accept allowed -> no shift; one in seven allowed -> no class shift
    assert mlp.calibration_shifts(out, y, 0.3, 0.15) == (0.0, 0.0)
    # a bar no grid value meets takes the largest grid value
    out2 = out.copy()
    out2[0, 0] = 100.0
    assert mlp.calibration_shifts(out2, y, 0.0, 1.0)[0] == 64.0
    # BF16 application: b3[0] - da and b3[1..3] + dc, rounded to FP32 then BF16
    bits = mlp.bf16_bits(np.zeros(mlp.N_PARAMS))
    new = mlp.apply_shifts(bits, 0.5, 0.25)
    vals = mlp.from_bf16_bits(new)
    assert (vals[5248:5252] == [-0.5, 0.25, 0.25, 0.25]).all() and (vals[:5248] == 0).all()
