"""GPU learned form: the BF16 network kernels against the oracle network, the
gated traversal against the oracle's gated tree code, and the measured pair
errors against the oracle's, through the C ABI.

Bars: network outputs and gradients within the BF16 tolerance of the FP64
oracle (and closer to the oracle run at the kernels' activation precision);
without a model the learned context is bitwise the fixed-degree method; with
a rule network the lists and their degree classes equal the oracle's and the
FP64 velocity is within 1e-10; pair errors within 1e-9 of the scale.
"""

import sys

import numpy as np
import pytest

import synthetic as S
from oracle import learned as OL
from oracle import mlp as OM

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def bf16_tensor(vals):
    """BF16 device tensor holding exactly OM.bf16_round(vals)."""
    bits = OM.bf16_bits(vals).astype(np.int16)
    return dev(bits).view(torch.bfloat16)


def _rows(n, seed):
    rng = np.random.default_rng(seed)
    x = np.zeros((n, 16))
    x[:, :12] = rng.uniform(-1, 1, (n, 12))
    y = (rng.uniform(size=(n, 4)) < 0.5).astype(np.float32)
    return OM.bf16_round(x), y


def _params(seed):
    th = OM.init_params(seed)
    th[OM.SLICES["b1"][0]:OM.SLICES["b1"][0] + 64] = np.random.default_rng(seed + 1).normal(0, 0.1, 64)
    th[OM.SLICES["b2"][0]:OM.SLICES["b2"][0] + 64] = np.random.default_rng(seed + 2).normal(0, 0.1, 64)
    return OM.bf16_round(th)


def _passthrough_params():
    """Parameters whose network outputs equal input features 0..3 exactly, in
    BF16 on the GPU and in FP64 in the oracle, for features on the grid k/16
    in [-4, 4]: unit weights route feature k through hidden unit k (shifted
    by +8 so the ReLUs pass it, every value a BF16 number), b3 = -8."""
    p = {k: np.zeros(s) for k, (_, s) in OM.SLICES.items()}
    for k in range(4):
        p["W1"][k, k] = 1.0
        p["b1"][k] = 8.0
        p["W2"][k, k] = 1.0
        p["W3"][k, k] = 1.0
    p["b3"][:] = -8.0
    return OM.pack(p)


def _cos(a, b):
    return float((a * b).sum() / np.sqrt((a * a).sum() * (b * b).sum()))


def test_forward_matches_oracle(stc_lib):
    th = _params(1)
    x, _ = _rows(1003, 2)
    out = stc_lib.mlp_forward(bf16_tensor(x), bf16_tensor(th)).cpu().numpy()
    ref_k, _ = OM.forward(th, x, act_round=OM.bf16_round)   # the kernels' activation precision
    ref, _ = OM.forward(th, x)                               # plain FP64
    scale = np.abs(ref).max()
    assert np.abs(out - ref_k).max() / scale < 1e-5
    assert np.abs(out - ref).max() / scale < 2e-2


@pytest.mark.parametrize("use_index", [False, True])
def test_gradient_matches_oracle(stc_lib, use_index):
    th = _params(3)
    x, y = _rows(2000, 4)
    idx = np.random.default_rng(5).choice(2000, 777, replace=False).astype(np.int32) if use_index else None
    g, loss = stc_lib.mlp_grad(bf16_tensor(x), dev(y), bf16_tensor(th), index=None if idx is None else dev(idx))
    g, loss = g.cpu().numpy(), float(loss.cpu().numpy()[0])
    xs, ys = (x[idx], y[idx]) if use_index else (x, y)
    gk = OM.grad(th, xs, ys, act_round=OM.bf16_round)
    g64 = OM.grad(th, xs, ys)
    assert abs(loss - OM.loss(th, xs, ys, act_round=OM.bf16_round)) < 1e-5 * abs(loss)
    for name, (o, sh) in OM.SLICES.items():
        n = int(np.prod(sh))
        a, bk, b = g[o:o + n], gk[o:o + n], g64[o:o + n]
        say(f"  {name}: cos(kernel precision) {_cos(a, bk):.6f} cos(FP64) {_cos(a, b):.6f}")
        assert _cos(a, bk) > 0.9999, name
        assert np.abs(a - bk).max() <= 2e-3 * np.abs(bk).max() + 1e-9, name
        assert _cos(a, b) > 0.999, name


def test_training_learns_a_rule(stc_lib):
    """Labels from a fixed rule on two features; GPU training (forward,
    backward, Adam) must reach a low loss and a high accuracy."""
    rng = np.random.default_rng(7)
    n = 20000
    x = np.zeros((n, 16))
    x[:, :12] = rng.uniform(0, 1, (n, 12))
    x = OM.bf16_round(x)
    y = np.zeros((n, 4), dtype=np.float32)
    y[:, 0] = x[:, 6] < 0.6
    for k in range(3):
        y[:, k + 1] = y[:, 0] * (x[:, 4] > 0.2 + 0.2 * k)
    master = dev(OM.init_params(9).astype(np.float32))
    params, losses = stc_lib.mlp_train(bf16_tensor(x), dev(y), master, epochs=20, batch=1024, lr=3e-3, seed=1)
    losses = losses.cpu().numpy()
    say(f"  loss first {losses[0]:.4f} last {losses[-20:].mean():.4f}")
    assert losses[-20:].mean() < 0.25 * losses[0]
    out = stc_lib.mlp_forward(bf16_tensor(x), params).cpu().numpy()
    acc, cls = OM.decide(out)
    assert (acc == (y[:, 0] > 0)).mean() > 0.97
    ok = y[:, 0] > 0
    assert (cls[ok] == y[ok, 1:].sum(1)).mean() > 0.9
    # the BF16 copy is the rounded master copy
    assert np.array_equal(OM.bf16_round(master.cpu().numpy()), params.float().cpu().numpy())


def _case(level=4, seed=7):
    x = S.icosahedral_grid(level) @ S.random_rotation(seed).T
    z = S.rossby_haurwitz(x, 4) + S.gaussian_vortex(x, seed=seed, amplitude=1e-4)
    return x, z, S.uniform_areas(len(x))


KW = dict(theta=0.6, n_crit=16)


def test_without_model_equals_fixed_degree(stc_lib):
    x, z, a = _case()
    say(f"learned vs fixed degree N={len(x)}")
    for precision in ("fp64", "fp32"):
        cl = stc_lib.Context(len(x), degree=10, precision=precision, denominator="dist2", learned=True,
                             theta_max=0.85, **KW)
        cp = stc_lib.Context(len(x), degree=10, precision=precision, denominator="dist2", max_level=cl.max_level,
                             **KW)
        ul = cl.velocity(dev(x), dev(z), dev(a)).cpu().numpy()
        up = cp.velocity(dev(x), dev(z), dev(a)).cpu().numpy()
        assert np.array_equal(ul, up), precision
        for k in ("PP", "PC", "CP", "CC"):
            assert np.array_equal(cl.copy_list(k), cp.copy_list(k)), k
        assert (cl.copy_list_classes("CC") == 3).all()
        assert cl.list_counts() == cp.list_counts()
        cl.close()
        cp.close()


def _rule_params(taus):
    """A network whose decisions are a rule on feature 6, (r_t + r_s) / R:
    accept iff f6 < tau0, degree class = #{k : f6 > tau_k}; every weight a
    power of two and every hidden value of one sign, so the decisions do not
    depend on rounding."""
    p = {"W1": np.zeros((12, 64)), "b1": np.zeros(64), "W2": np.zeros((64, 64)), "b2": np.zeros(64),
         "W3": np.zeros((64, 4)), "b3": np.zeros(4)}
    for j, tau in enumerate(taus):
        p["W1"][6, 2 * j], p["b1"][2 * j] = 1.0, -tau          # relu(f6 - tau_j)
        p["W1"][6, 2 * j + 1], p["b1"][2 * j + 1] = -1.0, tau  # relu(tau_j - f6)
    for i in range(8):
        p["W2"][i, i] = 1.0
    p["W3"][1, 0], p["W3"][0, 0] = 64.0, -64.0                 # o0 = 64 (tau0 - f6)
    for k in (1, 2, 3):
        p["W3"][2 * k, k], p["W3"][2 * k + 1, k] = 64.0, -64.0  # ok = 64 (f6 - tau_k)
    return OM.pack(p)


def _gap_thresholds(f6):
    """Four BF16 thresholds strictly between observed feature values."""
    vals = np.unique(f6)
    out = []
    for q in (0.8, 0.2, 0.45, 0.65):
        i = int(q * (len(vals) - 1))
        lo, hi = vals[i], vals[min(i + 1, len(vals) - 1)]
        cand = OM.bf16_round(np.array([(lo + hi) / 2]))[0]
        if not (lo < cand < hi):   # adjacent BF16 values: move to the next gap
            j = i + 1
            while j + 1 < len(vals):
                lo, hi = vals[j], vals[j + 1]
                cand = OM.bf16_round(np.array([(lo + hi) / 2]))[0]
                if lo < cand < hi:
                    break
                j += 1
        assert lo < cand < hi
        out.append(float(cand))
    return out


def test_rule_network_lists_and_velocity_match_oracle(stc_lib):
    x, z, a = _case()
    say(f"rule network N={len(x)}")
    # the oracle's own features fix the thresholds
    probe = OL.LearnedTree(x, z, a, theta_max=0.85, degree=8, den="dist2", **KW)
    taus = _gap_thresholds(probe.features[:, 6])
    th = _rule_params(taus)

    def rule(F):
        f6 = F[:, 6]
        return f6 < taus[0], (f6[:, None] > np.array(taus[1:])[None, :]).sum(1)

    ot = OL.LearnedTree(x, z, a, theta_max=0.85, degree=8, den="dist2", decide=rule, max_level=probe.max_level,
                        **KW)
    assert ot.accept.any() and not ot.accept.all()
    assert len(np.unique(ot.cls[ot.accept])) >= 3
    cl = stc_lib.Context(len(x), degree=8, precision="fp64", denominator="dist2", learned=True, theta_max=0.85,
                         max_level=probe.max_level, **KW)
    model = bf16_tensor(th)
    cl.set_model(model)
    u = cl.velocity(dev(x), dev(z), dev(a)).cpu().numpy()
    pairs, out, feat = cl.copy_candidates()
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    assert np.array_equal(pairs[order], ot.candidates)
    gf = OM.from_bf16_bits(feat[order])
    assert np.array_equal(gf[:, 6], ot.features[:, 6])
    # the other features: equal up to one BF16 step (transcendentals may round apart)
    assert (np.abs(gf - ot.features) <= np.abs(ot.features) * 2 ** -7 + 1e-30).all()
    for k in ("PP", "PC", "CP", "CC"):
        got = cl.copy_list(k)
        cls = cl.copy_list_classes(k)
        o = np.lexsort((cls, got[:, 1], got[:, 0]))
        assert np.array_equal(got[o], ot.lists[k]), k
        assert np.array_equal(cls[o], ot.classes[k]), k
    ref = ot.velocity()
    assert np.abs(u - ref).max() / np.abs(ref).max() < 1e-10
    cl.close()


def test_pair_errors_and_labels_match_oracle(stc_lib):
    x, z, a = _case(level=4, seed=3)
    say(f"pair errors N={len(x)}")
    ot = OL.LearnedTree(x, z, a, theta_max=0.8, degree=10, den="dist2", theta=0.6, n_crit=32)
    E = ot.pair_errors()
    tol = float(np.median(E[:, 2]))
    cl = stc_lib.Context(len(x), degree=10, precision="fp64", denominator="dist2", learned=True, theta_max=0.8,
                         theta=0.6, n_crit=32, max_level=ot.max_level)
    cl.tree_build(dev(x))
    cl.upward(dev(z), dev(a))
    feat, lab, err, n = cl.learned_samples(tol, 4 * len(ot.candidates) + 16)
    pairs, _, _ = cl.copy_candidates()
    assert n == len(ot.candidates)
    o = np.lexsort((pairs[:, 1], pairs[:, 0]))
    assert np.array_equal(pairs[o], ot.candidates)
    err = err.cpu().numpy()[o]
    scale = np.abs(ot.q).sum()
    assert np.abs(err - E).max() < 1e-9 * scale
    lab = lab.cpu().numpy()[o]
    want = OL.labels_from_errors(E, tol)
    clear = (np.abs(E - tol) > 1e-6 * tol).all(1)
    assert clear.mean() > 0.95
    assert np.array_equal(lab[clear], want[clear])
    fb = feat.view(torch.int16).cpu().numpy().view(np.uint16)
    assert np.array_equal(OM.from_bf16_bits(fb[o][:, 6]), ot.features[:, 6])
    cl.close()


def _ms_per_eval(ctx, xd, zd, ad, reps=5):
    out = torch.empty((xd.shape[0], 3), dtype=torch.float64, device="cuda")
    ctx.velocity(xd, zd, ad, out=out)
    ctx.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.velocity(xd, zd, ad, out=out)
    e1.record()
    torch.cuda.synchronize()
    ctx.sync()
    return e0.elapsed_time(e1) / reps


def test_trained_gate_gains_over_fixed_degree(stc_lib):
    """The learned form end to end, trained as configured: 2e6 samples
    labelled by the tree code's own measured pair errors at N = 163842
    (seeded inputs taken until that many), GPU training and calibration,
    then the evaluation at N = 2621442 (Gaussian vortex pair on a
    Rossby-Haurwitz background): rel-L2 error <= 1e-6 against the FP64
    direct sum on 4096 seeded targets, within 1e-6 of the fixed-degree-10
    FP64 tree (the reference), and fewer kernel evaluations than both that tree
    and the fastest fixed-degree FP32 setting that meets 1e-6 on this input
    (theta 0.8, d = 10).  Wall-clock time of the learned form and of that
    FP32 setting is measured (best of three rounds of five evaluations,
    alternating) and reported; the learned form must not be slower."""
    from paper_2401_07361_amd import gate_training as G
    from oracle import metrics

    def inputs():
        for k in range(64):
            x, z, a = S.make_gate_training_input(k)
            yield dev(x), dev(z), dev(a)

    F, Y = G.collect(inputs(), 3e-8, theta=0.7, theta_max=0.9, log=say, max_samples=2_000_000)
    params, losses = G.train(F, Y, epochs=8, batch=4096, lr=2e-3)
    ln = losses.cpu().numpy()
    say(f"  {F.shape[0]} samples, loss {ln[0]:.3f} -> {ln[-50:].mean():.3f}")
    assert ln[-50:].mean() < 0.2 * ln[0]
    params, da, dc = G.calibrate(F, Y, params, 1e-3, 1e-3)
    wl = S.make_workload("gvpair_l9")
    x, z, a, sub = wl["x"], wl["zeta"], wl["area"], wl["subset"]
    n = len(x)
    xd, zd, ad = dev(x), dev(z), dev(a)
    ud = stc_lib.direct(xd, zd, ad, targets=dev(sub), denominator="dist2").cpu().numpy()
    ref = stc_lib.Context(n, theta=0.7, degree=10, n_crit=64, precision="fp64", denominator="dist2")
    uj = ref.velocity(xd, zd, ad).cpu().numpy()
    _, ej = ref.list_counts()
    ref.close()
    ctx = stc_lib.Context(n, theta=0.7, theta_max=0.9, degree=10, n_crit=64, precision="fp32", denominator="dist2",
                          learned=True)
    ctx.set_model(params)
    ul = ctx.velocity(xd, zd, ad).cpu().numpy()
    _, el = ctx.list_counts()
    cls = {k: np.bincount(ctx.copy_list_classes(k), minlength=4).tolist() for k in ("PC", "CP", "CC")}
    fixed = stc_lib.Context(n, theta=0.8, degree=10, n_crit=64, precision="fp32", denominator="dist2")
    uf = fixed.velocity(xd, zd, ad).cpu().numpy()
    _, ef = fixed.list_counts()
    ms_learned, ms_fixed = float("inf"), float("inf")
    for _ in range(3):
        ms_learned = min(ms_learned, _ms_per_eval(ctx, xd, zd, ad))
        ms_fixed = min(ms_fixed, _ms_per_eval(fixed, xd, zd, ad))
    ctx.close()
    fixed.close()
    e_fixed = metrics.rel_l2_velocity(uf[sub], ud, a[sub])
    e_direct = metrics.rel_l2_velocity(ul[sub], ud, a[sub])
    e_ref = metrics.rel_l2_velocity(ul, uj, a)
    say(f"  N={n}: E vs direct {e_direct:.3e}, vs FP64 fixed-degree tree {e_ref:.3e}; evaluations "
        f"{sum(el.values()) / 1e9:.3f}e9 vs {sum(ej.values()) / 1e9:.3f}e9; classes {cls}")
    say(f"  against fixed FP32 theta 0.8 d 10 (E {e_fixed:.3e}): evaluations {sum(el.values()) / 1e9:.3f}e9 vs "
        f"{sum(ef.values()) / 1e9:.3f}e9, {ms_learned:.3f} ms vs {ms_fixed:.3f} ms per evaluation "
        f"({'faster' if ms_learned < ms_fixed else 'slower'} by {abs(1 - ms_learned / ms_fixed) * 100:.1f}%)")
    assert e_direct <= 1e-6
    assert e_ref <= 1e-6
    assert e_fixed <= 1e-6
    assert sum(el.values()) < 0.6 * sum(ej.values())
    assert sum(el.values()) < 0.7 * sum(ef.values())
    assert sum(1 for c in cls["CC"] if c > 0) >= 3   # the network uses several degrees
    assert ms_learned < ms_fixed


def test_learned_arguments_are_checked(stc_lib):
    with pytest.raises(stc_lib.StcError):        # one member only
        stc_lib.Context(1000, members=2, learned=True, degree=10, denominator="dist2")
    with pytest.raises(stc_lib.StcError):        # degree must be a class degree
        stc_lib.Context(1000, learned=True, degree=7, denominator="dist2")
    with pytest.raises(stc_lib.StcError):        # theta_max below theta
        stc_lib.Context(1000, learned=True, degree=10, theta=0.7, theta_max=0.5, denominator="dist2")
    plain = stc_lib.Context(1000, degree=10)
    with pytest.raises(stc_lib.StcError):        # no learned traversal in a plain context
        plain.set_model(bf16_tensor(np.zeros(stc_lib.mlp_param_count())))
    plain.close()
    cl = stc_lib.Context(1000, learned=True, degree=10, denominator="dist2")
    p = bf16_tensor(np.zeros(stc_lib.mlp_param_count() + 8))
    with pytest.raises(stc_lib.StcError):        # misaligned parameters
        cl.set_model(p[1:1 + stc_lib.mlp_param_count()])
    cl.close()


def test_forcing_applies_to_the_learned_form(stc_lib):
    """The vorticity forcing acts on the charges, upstream of the gating: a
    learned context without a network equals the fixed-degree context under
    the same forcing, bitwise, and the forcing changes the result."""
    x, z, a = _case()
    om, lat1, tp, tf = 2.0 * np.pi, np.pi / 3.0, 4.0, 15.0
    say(f"learned form with forcing N={len(x)}")
    cl = stc_lib.Context(len(x), degree=10, precision="fp32", denominator="dist2", learned=True, theta_max=0.85,
                         **KW)
    cp = stc_lib.Context(len(x), degree=10, precision="fp32", denominator="dist2", max_level=cl.max_level, **KW)
    u0 = cp.velocity(dev(x), dev(z), dev(a)).cpu().numpy()
    for c in (cl, cp):
        c.set_forcing(2, om, lat1, tp, tf, time=7.0)
    ul = cl.velocity(dev(x), dev(z), dev(a)).cpu().numpy()
    up = cp.velocity(dev(x), dev(z), dev(a)).cpu().numpy()
    assert np.array_equal(ul, up)
    assert np.abs(up - u0).max() > 1e-3 * np.abs(u0).max()
    cl.close()
    cp.close()


@pytest.mark.parametrize("n,fa,uc", [(20000, 0.05, 0.02), (5000, 0.001, 0.001), (3000, 1.0, 1.0)])
def test_calibration_matches_oracle(stc_lib, n, fa, uc):
    """stc_mlp_calibrate against the oracle's calibration on outputs both
    sides compute exactly (pass-through network, features on a 1/16 grid, so
    no output ties a grid value): the same shifts and bitwise the same
    calibrated BF16 parameters."""
    say(f"calibration n={n} fa={fa} uc={uc}")
    rng = np.random.default_rng(n)
    x = np.zeros((n, 16))
    x[:, :4] = rng.integers(-64, 65, (n, 4)) / 16.0
    y = np.zeros((n, 4), dtype=np.float32)
    y[:, 0] = rng.uniform(size=n) < 0.6
    steps = rng.integers(0, 4, n)
    for k in range(3):
        y[:, k + 1] = (y[:, 0] > 0) & (steps > k)
    th = _passthrough_params()
    out_o, _ = OM.forward(th, x)
    assert np.array_equal(out_o, x[:, :4])
    out_g = stc_lib.mlp_forward(bf16_tensor(x), bf16_tensor(th)).cpu().numpy()
    assert np.array_equal(out_g.astype(np.float64), x[:, :4])
    da, dc = OM.calibration_shifts(out_o, y, fa, uc)
    newp, shifts = stc_lib.mlp_calibrate(bf16_tensor(x), dev(y), bf16_tensor(th), fa, uc)
    got = shifts.cpu().numpy()
    assert got[0] == pytest.approx(da, rel=1e-15, abs=0) and got[1] == pytest.approx(dc, rel=1e-15, abs=0)
    ref_bits = OM.apply_shifts(OM.bf16_bits(th), da, dc)
    got_bits = newp.view(torch.int16).cpu().numpy().astype(np.uint16)
    assert np.array_equal(got_bits, ref_bits)


def test_label_scale_matches_numpy(stc_lib):
    rng = np.random.default_rng(3)
    u = rng.standard_normal((100003, 3)) * 1e-5
    say("label scale")
    got = float(stc_lib.label_scale(dev(u)).item())
    ref = 4.0 * np.pi * np.sqrt((u * u).sum(1).mean())
    assert got == pytest.approx(ref, rel=1e-13)
