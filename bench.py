"""Benchmark: particle velocity evaluations per second of the spherical tree
code at N = 655362 (icosahedron refined 8 times), Gaussian vortex of width 0.1
plus 1e-3 uniform noise, A = 4 pi / N, precision form (FP32 kernel sums with
the |x - y|^2 / 2 denominator, FP64 proxy charges), accuracy checked against
the FP64 direct sum on 4096 seeded targets.

One step = one full velocity evaluation (tree build, upward pass, traversal,
near and far field, output) on inputs already resident in HBM.  Prints one
JSON line.  Single GPU only.

``--workload learned`` times the learned form: the gating network is trained
on the GPU from six seeded N = 163842 inputs (samples labelled by the tree
code's measured pair errors), then one step is a learned-form evaluation at
N = 2621442 (Gaussian vortex pair on a Rossby-Haurwitz background), checked
against the FP64 direct sum and the fixed-degree-10 FP64 tree, and set
beside the fixed-degree method in FP32 and FP64.

``--workload ensemble`` times the batching form instead: 48 seeded members
(levels 5-7, 3.87e6 particles in total, random rotations, RH waves of
wavenumber 3-5 plus a Gaussian bump), all members in one launch per phase,
against the same members evaluated one context after the other; it also
times graph-captured RK4 steps of the whole ensemble.

``--workload rk4`` times graph-captured RK4 steps of the Rossby-Haurwitz wave
at N = 163842; ``--workload rh10d`` runs that wave for its configured ten days
(480 steps) in FP64 and FP32 and reports the phase against the closed form,
the circulation drift and E_N, with tree and resolution controls; ``--workload ssw`` those of the forced polar-vortex collapse
(Sec. 4.4) at N = 163842, d = 6, theta = 0.7; ``--workload stream`` the stream
function (logarithmic kernel) on the headline workload and setting;
``--workload plain`` the plain FP64 method (theta 0.7, d 8) at N = 10242.
"""

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Benchmark setting: the fastest (theta, degree, N_T) whose error on this
# workload stays about a factor 2 below the 1e-6 bar (E = 5.0e-7).
BENCH_THETA = 0.8
BENCH_DEGREE = 10
BENCH_N_CRIT = 64

FP32_FLOPS = 16   # per |x-y|^2/2 kernel evaluation: 3 sub, |d|^2 5, div 1, *q 1, 3 fma 6
FP64_FLOPS = 17   # per 1 - x.y evaluation with the (y - x) form: dot 5, 1- 1, div 1, *q 1, 3 sub, 3 fma 6
# Published MI355X peaks (vector): FP32 157.3 TFLOP/s (packed FP32 instructions), FP64 78.6 TFLOP/s.
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
# What the library's FP32 code can issue: it is built without packed FP32 instructions, so FP32 and FP64
# FMAs both issue 64 lanes per CU per clock: 256 CU x 64 lanes x 2 flop x 2.4 GHz.
PEAK_VALU_TFLOPS = 78.6
COPY_BYTES = 256 << 20    # calibration copy: bytes read = bytes written
# evaluation kernels: phase name -> (kernel, lists it evaluates, recorded HBM traffic summary)
EVAL_KERNELS = {
    "near": ("k_near (PP + PC)", ("PP", "PC"), os.path.join(ROOT, "profiles", "k_near_gv_l8_hbm_traffic.md")),
    "far_targets": ("k_far_targets (CP + CC)", ("CP", "CC"),
                    os.path.join(ROOT, "profiles", "k_far_targets_gv_l8_hbm_traffic.md")),
}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("k_eval.hip", "common.hpp", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2401_07361_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(config_tag, path):
    """HBM bytes per launch of one evaluation kernel from the committed counter
    summary at `path`, if it was taken on the current kernel source and the
    same configuration."""
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].strip().split(": ", 1)
            rec[k] = v.strip("` ")
    if rec.get("kernel_source_hash") != kernel_source_hash() or rec.get("config") != config_tag:
        return None
    try:
        return int(rec["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


_G = {}


def _oracle_worker(idx):
    from oracle import direct
    fn = direct.stream_function if _G["stream"] else direct.velocity
    return fn(_G["x"], _G["z"], _G["a"], targets=idx, den=_G["den"])


def cpu_baseline(x, z, a, subset, budget_s=15.0, den="dot", what="the 4096 seeded targets", stream=False):
    """The oracle's direct sum (O(N) per target) timed on the host cores over a
    bounded sample of the target subset (the stream function's with stream)."""
    from oracle import direct
    # a one-GPU job is allotted 16 host CPUs (more visible CPUs are shared
    # with other jobs), so the pool takes at most 16 processes
    visible = len(os.sched_getaffinity(0))
    cores = min(visible, 16)
    _G.update(x=x, z=z, a=a, den=den, stream=stream)
    fn = direct.stream_function if stream else direct.velocity
    t0 = time.perf_counter()
    probe = fn(x, z, a, targets=subset[:8], den=den)
    per_target = (time.perf_counter() - t0) / 8
    m = int(min(len(subset), max(cores * 8, budget_s * cores / per_target)))
    m = max(8, (m // cores) * cores) if m >= cores else m
    sample = subset[:m]
    chunks = np.array_split(sample, cores * 4)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        parts = pool.map(_oracle_worker, chunks)
    dt = time.perf_counter() - t0
    u = np.concatenate(parts)
    return dict(value=m / dt, unit="velocity evals/s", cores=cores, cpus_visible=visible, kind="oracle",
                sample=f"{m} of {what}, all {len(x)} sources, FP64 direct "
                       f"{'stream function' if stream else 'sum'}, "
                       f"{dt:.1f} s wall"), sample, u


def roofline(evals, kern_ms, precision, flops=None, config_tag=None):
    """ALU roofline of the evaluation kernels: an entry per kernel (k_near:
    PP + PC, k_far_targets: CP + CC) from exact list evaluation counts and the
    kernel's average duration measured with HIP events on the library stream
    inside the timed region; the dominant kernel (longest per launch) is the
    returned object, the other under "kernels".  `peak` is the published
    vector peak of the precision; FP32 also reports the fraction of the
    78.6 TFLOP/s the library's non-packed FP32 code can issue."""
    fl = flops if flops is not None else (FP32_FLOPS if precision == "fp32" else FP64_FLOPS)
    peak = PEAK_FP32_TFLOPS if precision == "fp32" else PEAK_FP64_TFLOPS
    entries = []
    for ph, (name, lists, tfile) in EVAL_KERNELS.items():
        if ph not in kern_ms:
            continue
        ev = int(sum(evals[k] for k in lists))
        ms = kern_ms[ph]
        achieved = ev * fl / (ms / 1e3) / 1e12
        e = dict(bound="alu", achieved=round(achieved, 3), peak=peak, unit="TFLOP/s", frac=round(achieved / peak, 4),
                 traffic=None, kernel=name, kernel_ms=round(ms, 4), kernel_evals_per_launch=ev, flops_per_eval=fl)
        if precision == "fp32":
            e["valu_issue_ceiling"] = PEAK_VALU_TFLOPS
            e["frac_of_valu_issue_ceiling"] = round(achieved / PEAK_VALU_TFLOPS, 4)
        if config_tag is not None:
            e["traffic"] = recorded_traffic(config_tag, tfile)
            e["traffic_source"] = ("recorded: " + os.path.relpath(tfile, ROOT)) if e["traffic"] is not None else None
        entries.append(e)
    entries.sort(key=lambda e: -e["kernel_ms"])
    top = dict(entries[0])
    top["kernels"] = entries
    return top


# the fastest setting whose worst member stays below 1e-6 (5.1e-7 on 256 targets per member;
# theta 0.7, d 8 reaches only 3.7e-6)
ENS_THETA, ENS_DEGREE, ENS_N_CRIT = 0.8, 10, 64


def ensemble_member_errors(stc, x, z, a, off, u, area_h, targets=256):
    """Area-weighted relative L2 error of each member's velocity u against its
    FP64 direct sum (|x - y|^2 / 2) at `targets` seeded particles."""
    import torch
    un = u.cpu().numpy()
    errs = []
    for m in range(len(off) - 1):
        lo, hi = int(off[m]), int(off[m + 1])
        tg = np.random.default_rng(100 + m).choice(hi - lo, min(targets, hi - lo), replace=False)
        ref = stc.direct(x[lo:hi], z[lo:hi], a[lo:hi], targets=torch.from_numpy(tg.astype(np.int64)).cuda(),
                         denominator="dist2").cpu().numpy()
        w = area_h[lo:hi][tg][:, None]
        errs.append(float(np.sqrt((w * (un[lo:hi][tg] - ref) ** 2).sum() / (w * ref ** 2).sum())))
    return errs


def bench_ensemble(args):
    import torch
    import synthetic as S
    from paper_2401_07361_amd import stc

    ens = S.make_ensemble()
    off = ens["offsets"]
    M, N = len(off) - 1, int(off[-1])
    log(f"workload ensemble members={M} N={N} theta={ENS_THETA} d={ENS_DEGREE} n_crit={ENS_N_CRIT} fp32")
    x, z, a = (torch.from_numpy(ens[k]).cuda() for k in ("x", "zeta", "area"))
    out = torch.empty((N, 3), dtype=torch.float64, device="cuda")
    kw = dict(theta=ENS_THETA, degree=ENS_DEGREE, n_crit=ENS_N_CRIT, precision="fp32", denominator="dist2")
    ctx = stc.Context(N, members=M, n_max_member=int(np.diff(off).max()), **kw)
    ctx.velocity_batched(x, z, a, off, out=out)
    shape = ctx.autotune(repeats=3)
    log(f"autotuned launch shape {shape}")
    ms, kern_ms, phase_ms = _timed(ctx, lambda: ctx.velocity_batched(x, z, a, off, out=out), args.steps,
                                   args.warmup)
    counts, evals = ctx.list_counts()
    log(f"batched: {ms:.3f} ms per ensemble evaluation; phases {phase_ms}")
    # accuracy: 256 seeded targets per member against that member's FP64 direct sum
    errs0 = ensemble_member_errors(stc, x, z, a, off, out, ens["area"])
    worst = max(errs0)
    # the same members one context at a time (one launch sequence per member)
    singles = [stc.Context(int(off[m + 1] - off[m]), max_level=ctx.max_level, **kw) for m in range(M)]
    views = [(x[int(off[m]):int(off[m + 1])], z[int(off[m]):int(off[m + 1])], a[int(off[m]):int(off[m + 1])],
              out[int(off[m]):int(off[m + 1])]) for m in range(M)]
    for c, (xv, zv, av, ov) in zip(singles, views):
        c.velocity(xv, zv, av, out=ov)
    torch.cuda.synchronize()
    seq_steps = max(1, args.steps // 4)
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(seq_steps):
        for c, (xv, zv, av, ov) in zip(singles, views):
            c.velocity(xv, zv, av, out=ov)
    t1.record()
    torch.cuda.synchronize()
    ms_seq = t0.elapsed_time(t1) / seq_steps
    for c in singles:
        c.close()
    log(f"one member at a time: {ms_seq:.3f} ms per ensemble evaluation")
    # the configured run: 24 graph-captured RK4 steps of the whole ensemble
    # (dt = 1800 s) from the initial state, then every member's error at its
    # final state
    xr, zr = x.clone(), z.clone()
    ctx.rk4_batched(xr, zr, a, off, ens["dt"], S.OMEGA_EARTH_S, 1)   # captures the step graph
    torch.cuda.synchronize()
    xr.copy_(x)
    zr.copy_(z)
    rk_steps = ens["steps"]
    t0.record()
    ctx.rk4_batched(xr, zr, a, off, ens["dt"], S.OMEGA_EARTH_S, rk_steps)
    t1.record()
    torch.cuda.synchronize()
    ms_rk = t0.elapsed_time(t1) / rk_steps
    ctx.sync()
    log(f"rk4 step (4 evaluations, one graph): {ms_rk:.3f} ms over {rk_steps} steps")
    ctx.velocity_batched(xr, zr, a, off, out=out)
    errs = ensemble_member_errors(stc, xr, zr, a, off, out, ens["area"])
    log(f"after {rk_steps} steps: worst member E {max(errs):.3e}, median {np.median(errs):.3e}")
    ctx.close()
    roof = roofline(evals, kern_ms, "fp32")
    m0 = ens["members"][0]
    cb = None
    if not args.no_cpu:
        log("cpu baseline (oracle direct sum, member 0, bounded target sample)")
        tg = np.random.default_rng(100).choice(len(m0["x"]), 64, replace=False)
        cb, _, _ = cpu_baseline(m0["x"], m0["zeta"], m0["area"], tg, budget_s=8.0, den="dist2",
                                what=f"64 seeded targets of member 0 (N={len(m0['x'])})")
    result = dict(
        metric="ensemble particle velocity evals/s (48 members, one launch per phase)",
        value=N / (ms / 1e3), unit="velocity evals/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(ms, 4), higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
        data="synthetic",
        config=dict(workload="ensemble (48 members, icosahedral levels 5-7, RH n=3-5 + Gaussian bump)",
                    members=M, N=N, theta=ENS_THETA, degree=ENS_DEGREE, n_crit=ENS_N_CRIT,
                    max_level=int(ctx.max_level), precision="fp32", denominator="dist2",
                    launch_shape=list(shape), worst_member_rel_l2_err_vs_fp64_direct=float(f"{worst:.3e}"),
                    rk4_steps=int(ens["steps"]),
                    after_rk4=dict(worst_member_rel_l2_err=float(f"{max(errs):.3e}"),
                                   median_member_rel_l2_err=float(f"{np.median(errs):.3e}"),
                                   members_within_1e_6=int(sum(e <= 1e-6 for e in errs))),
                    lists=counts, kernel_evals=int(sum(evals.values())), phase_ms=phase_ms,
                    ms_one_member_at_a_time=round(ms_seq, 4), batching_speedup=round(ms_seq / ms, 3),
                    ms_per_rk4_step=round(ms_rk, 4)),
        roofline=roof,
    )
    if cb is not None:
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


# training: the configured 2e6 samples, from as many seeded N = 163842 inputs as it takes (about 64k
# candidate pairs each)
LEARNED = dict(theta=0.7, theta_max=0.9, degree=10, n_crit=64, tol_rel=3e-8, train_samples=2_000_000,
               max_inputs=64, epochs=8, batch=4096, lr=2e-3)


def _phase_breakdown(ctx, fn, reps=3):
    """Every phase of `reps` extra calls, with an event at each phase boundary
    (outside the timed region: each event adds a gap between kernels)."""
    ctx.set_timing(reps)
    for _ in range(reps):
        fn()
    ctx.sync()
    ph, k = ctx.phase_times()
    return {p: round(v / max(k, 1), 4) for p, v in ph.items()}


def _timed(ctx, fn, steps, warmup):
    """(ms per call over the timed region, {phase: ms per launch} of k_near and
    k_far_targets measured with events around those kernels only inside the
    timed region, phase breakdown)."""
    import torch
    for _ in range(warmup):
        fn()
    ctx.set_timing(steps, phases=["near", "far_targets"])
    torch.cuda.synchronize()
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(steps):
        fn()
    t1.record()
    torch.cuda.synchronize()
    ctx.sync()
    ph, k = ctx.phase_times()
    kern_ms = {p: ph[p] / max(k, 1) for p in ("near", "far_targets")}
    return t0.elapsed_time(t1) / steps, kern_ms, _phase_breakdown(ctx, fn)


def bench_learned(args):
    import torch
    import synthetic as S
    from paper_2401_07361_amd import stc, gate_training as G
    from oracle import metrics

    P = LEARNED
    t0 = time.perf_counter()

    def inputs():
        for k in range(P["max_inputs"]):
            yield tuple(torch.from_numpy(v).cuda() for v in S.make_gate_training_input(k))

    F, Y = G.collect(inputs(), P["tol_rel"], P["theta"], P["theta_max"], degree=P["degree"], n_crit=P["n_crit"],
                     log=log, max_samples=P["train_samples"])
    torch.cuda.synchronize()
    t_samples = time.perf_counter() - t0
    t1 = time.perf_counter()
    params, losses = G.train(F, Y, epochs=P["epochs"], batch=P["batch"], lr=P["lr"])
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    params, da, dc = G.calibrate(F, Y, params, 1e-3, 1e-3)
    ln = losses.cpu().numpy()
    log(f"{F.shape[0]} samples in {t_samples:.2f} s, {len(ln)} training steps in {t_train:.2f} s, "
        f"loss {ln[0]:.3f} -> {ln[-50:].mean():.3f}")
    wl = S.make_workload("gvpair_l9")
    x, z, a, sub = wl["x"], wl["zeta"], wl["area"], wl["subset"]
    n = len(x)
    xd, zd, ad = (torch.from_numpy(v).cuda() for v in (x, z, a))
    ud = stc.direct(xd, zd, ad, targets=torch.from_numpy(sub).cuda(), denominator="dist2").cpu().numpy()
    out = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    rows = {}

    def run(name, model=None, **kw):
        ctx = stc.Context(n, denominator="dist2", n_crit=P["n_crit"], **kw)
        if model is not None:
            ctx.set_model(model)
        ms, kern_ms_t, ph = _timed(ctx, lambda: ctx.velocity(xd, zd, ad, out=out), args.steps, args.warmup)
        cnt, ev = ctx.list_counts()
        if model is not None and kw.get("precision") == "fp32":
            pairs, _, _ = ctx.copy_candidates()
            rows["_near"] = (ev, kern_ms_t, len(pairs))
        u = out.cpu().numpy()
        rows[name] = dict(ms=round(ms, 4), rel_l2_err_vs_fp64_direct=float(f"{metrics.rel_l2_velocity(u[sub], ud, a[sub]):.3e}"),
                          kernel_evals=int(sum(ev.values())), phase_ms=ph)
        log(f"{name}: {ms:.3f} ms, E = {rows[name]['rel_l2_err_vs_fp64_direct']}, evals {sum(ev.values()) / 1e9:.3f}e9")
        ctx.close()
        return u

    uj = run("fixed_fp64_theta0.7_d10", theta=0.7, degree=10, precision="fp64")
    run("fixed_fp32_theta0.8_d10", theta=0.8, degree=10, precision="fp32")
    ul64 = run("learned_fp64", model=params, theta=P["theta"], theta_max=P["theta_max"], degree=P["degree"],
               precision="fp64", learned=True)
    ul = run("learned_fp32", model=params, theta=P["theta"], theta_max=P["theta_max"], degree=P["degree"],
             precision="fp32", learned=True)
    e_ref = metrics.rel_l2_velocity(ul, uj, a)
    roof_evals, roof_ms, n_cand = rows.pop("_near")
    # the network's forward pass over the candidates, timed on its own (MFMA, BF16)
    feats = F[: min(len(F), n_cand)] if n_cand <= len(F) else F
    fwd = torch.empty((feats.shape[0], 4), dtype=torch.float32, device="cuda")
    stc.mlp_forward(feats, params, out=fwd)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        stc.mlp_forward(feats, params, out=fwd)
    e1.record()
    torch.cuda.synchronize()
    mlp_ms = e0.elapsed_time(e1) / 20
    mlp_flops = 2.0 * (16 * 64 + 64 * 64 + 64 * 16) * feats.shape[0]   # padded MFMA shapes
    mlp_roof = dict(bound="mfma", achieved=round(mlp_flops / (mlp_ms / 1e3) / 1e12, 3), peak=2500.0,
                    unit="TFLOP/s", frac=round(mlp_flops / (mlp_ms / 1e3) / 1e12 / 2500.0, 6), traffic=None,
                    kernel="k_mlp_forward (BF16)", kernel_ms=round(mlp_ms, 4), rows=int(feats.shape[0]))
    log(f"network forward over {feats.shape[0]} rows: {mlp_ms:.4f} ms")
    r = rows["learned_fp32"]
    result = dict(
        metric="particle velocity evals/s at N=2621442 with learned degree/acceptance gating, rel-L2 err <=1e-6 vs FP64 direct sum",
        value=n / (r["ms"] / 1e3), unit="velocity evals/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=r["ms"], higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="gvpair_l9 (Gaussian vortex pair + RH n=4, icosahedral level 9)", N=n,
                    **{k: v for k, v in P.items()}, rel_l2_err_vs_fp64_direct=r["rel_l2_err_vs_fp64_direct"],
                    rel_l2_err_vs_fixed_degree_fp64_tree=float(f"{e_ref:.3e}"),
                    err_ok=bool(r["rel_l2_err_vs_fp64_direct"] <= 1e-6 and e_ref <= 1e-6),
                    training=dict(samples=int(F.shape[0]), seconds_samples=round(t_samples, 3),
                                  seconds_train=round(t_train, 3), steps=len(ln),
                                  loss_first=float(f"{ln[0]:.4f}"), loss_last=float(f"{ln[-50:].mean():.4f}"),
                                  calibration=dict(accept_shift=da, class_shift=dc)),
                    runs=rows, network_forward=mlp_roof),
        roofline=roofline(roof_evals, roof_ms, "fp32"),
    )
    if not args.no_cpu:
        log("cpu baseline (oracle direct sum, bounded target sample)")
        cb, _, _ = cpu_baseline(x, z, a, sub, budget_s=10.0, den="dist2")
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


def bench_rk4(args):
    import torch
    import synthetic as S
    from paper_2401_07361_amd import stc
    from oracle import metrics

    wl = S.make_workload("rh4_l7")
    x, z, a, sub = wl["x"], wl["zeta"], wl["area"], wl["subset"]
    n = len(x)
    dt, Om = wl["dt"], S.OMEGA_EARTH_S
    xd, zd, ad = (torch.from_numpy(v).cuda() for v in (x, z, a))
    ud = stc.direct(xd, zd, ad, targets=torch.from_numpy(sub).cuda(), denominator="dist2").cpu().numpy()
    runs = {}
    for prec in ("fp32", "fp64"):
        ctx = stc.Context(n, theta=wl["theta"], degree=wl["degree"], n_crit=64, precision=prec, denominator="dist2")
        u = ctx.velocity(xd, zd, ad)
        shape = ctx.autotune(repeats=5)  # launch shape for this size, used by the evaluations below
        log(f"{prec}: autotuned launch shape {shape}")
        err = metrics.rel_l2_velocity(u.cpu().numpy()[sub], ud, a[sub])
        ms_eval, kern_ms_t, ph = _timed(ctx, lambda: ctx.velocity(xd, zd, ad, out=u), args.steps, args.warmup)
        cnt, ev = ctx.list_counts()
        xs, zs = xd.clone(), zd.clone()
        ctx.rk4(xs, zs, ad, dt, Om, 1)   # captures the step graph
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        ctx.rk4(xs, zs, ad, dt, Om, args.steps)
        t1.record()
        torch.cuda.synchronize()
        ctx.sync()
        ms_step = t0.elapsed_time(t1) / args.steps
        runs[prec] = dict(ms_per_rk4_step=round(ms_step, 4), ms_per_evaluation=round(ms_eval, 4), launch_shape=shape,
                          rel_l2_err_vs_fp64_direct=float(f"{err:.3e}"), phase_ms=ph,
                          near=(ev, kern_ms_t))
        log(f"{prec}: {ms_step:.3f} ms per RK4 step (graph), {ms_eval:.3f} ms per evaluation, E = {err:.3e}")
        ctx.close()
    r = runs["fp32"]
    roof_evals, roof_ms = r.pop("near")
    runs["fp64"].pop("near")
    result = dict(
        metric="particle velocity evals/s in RK4 time stepping at N=163842 (4 evaluations per step, one HIP graph per step)",
        value=4 * n / (r["ms_per_rk4_step"] / 1e3), unit="velocity evals/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=r["ms_per_rk4_step"], higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="rh4_l7 (Rossby-Haurwitz n=4, icosahedral level 7, node-patch areas)", N=n,
                    theta=wl["theta"], degree=wl["degree"], n_crit=64, dt_seconds=dt, omega=Om, runs=runs),
        roofline=roofline(roof_evals, roof_ms, "fp32"),
    )
    if not args.no_cpu:
        log("cpu baseline (oracle direct sum, bounded target sample)")
        cb, _, _ = cpu_baseline(x, z, a, sub, budget_s=8.0, den="dist2", what="4096 seeded targets")
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


def rh_ten_day_run(stc, x0, z0, a, dt, Om, steps, precision, theta, degree, day_steps=48, log=None):
    """RK4 of the Rossby-Haurwitz wave (graph-captured steps, one sync per
    simulated day): final (x, zeta), the k = 4 phase after every day
    (unwrapped), and ms per step over the run."""
    import torch
    ctx = stc.Context(len(x0), theta=theta, degree=degree, n_crit=64, precision=precision, denominator="dist2")
    xd, zd, ad = (torch.from_numpy(v.copy()).cuda() for v in (x0, z0, a))
    phases = [rh_phase(x0, z0, a)]
    ms = 0.0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for day0 in range(0, steps, day_steps):
        k = min(day_steps, steps - day0)
        e0.record()
        ctx.rk4(xd, zd, ad, dt, Om, k)
        e1.record()
        torch.cuda.synchronize()
        ctx.sync()
        ms += e0.elapsed_time(e1)
        x, z = xd.cpu().numpy(), zd.cpu().numpy()
        phases.append(rh_phase(x, z, a))
        if log:
            log(f"  {precision} theta={theta} d={degree} N={len(x0)}: step {day0 + k} of {steps}")
    ctx.close()
    ph = np.unwrap(np.array(phases))
    return x, z, ph, ms / steps


def rh_phase(x, z, a, k=4):
    """Phase of the k-wave: arg sum A zeta z (x + i y)^k (the vorticity's
    projection on the wave's pattern); it advances by k nu t."""
    return float(np.angle(((x[:, 0] + 1j * x[:, 1]) ** k * x[:, 2] * z * a).sum()))


def bench_rh10d(args):
    """The Rossby-Haurwitz wave n = 4 at N = 163842 (icosahedral level 7,
    node-patch areas), RK4 with dt = 1800 s for 480 steps (10 days), plain
    FP64 and FP32 forms at theta 0.7, d 8.  Reported: phase after 10 days
    against the closed-form propagation (Sec. 4, Rossby-Haurwitz phase speed),
    relative circulation drift, E_N against the exact moved field, FP32 vs FP64
    differences, and two controls: a tighter tree (theta 0.4, d 12, FP64) to
    show the tree's approximation does not set the phase error, and the same
    run at level 6 (N = 40962) to show that the particle discretisation does."""
    import synthetic as S
    from paper_2401_07361_amd import stc
    from oracle import metrics

    wl = S.make_workload("rh4_l7")
    x0, z0, a = wl["x"], wl["zeta"], wl["area"]
    n, dt, steps = len(x0), wl["dt"], wl["steps"]
    Om = S.OMEGA_EARTH_S
    omega = K = 7.848e-6
    nu = (4 * (4 + 3) * omega - 2 * Om) / ((4 + 1) * (4 + 2))
    expected = np.degrees(nu * dt * steps)

    def report(tag, x, z, ph, ms, xs0, zs0, aa):
        shift = np.degrees(ph[-1] - ph[0]) / 4
        c, s_ = np.cos(-np.radians(shift)), np.sin(-np.radians(shift))
        R = np.array([[c, -s_, 0], [s_, c, 0], [0, 0, 1]])
        c2, s2 = np.cos(-nu * dt * steps), np.sin(-nu * dt * steps)
        R2 = np.array([[c2, -s2, 0], [s2, c2, 0], [0, 0, 1]])
        en_exact = metrics.rel_l2_scalar(z, S.rossby_haurwitz(x @ R2.T, 4, omega=omega, K=K), aa)
        en_moved = metrics.rel_l2_scalar(z, S.rossby_haurwitz(x @ R.T, 4, omega=omega, K=K), aa)
        drift = abs((z * aa).sum() - (zs0 * aa).sum()) / (np.abs(zs0) * aa).sum()
        r = dict(phase_deg=round(shift, 4), phase_rel_err=round((shift - expected) / expected, 5),
                 E_N_vs_exact=float(f"{en_exact:.4e}"), E_N_vs_field_at_measured_phase=float(f"{en_moved:.4e}"),
                 circulation_drift=float(f"{drift:.3e}"), ms_per_rk4_step=round(ms, 4),
                 daily_phase_deg=[round(v, 3) for v in np.degrees(ph - ph[0]) / 4])
        log(f"{tag}: phase {shift:.3f} deg (closed form {expected:.3f}), E_N {en_exact:.3e}, "
            f"drift {drift:.2e}, {ms:.3f} ms/step")
        return r

    runs = {}
    finals = {}
    for tag, prec, th, d in (("fp64", "fp64", 0.7, 8), ("fp32", "fp32", 0.7, 8),
                             ("fp64_theta0.4_d12", "fp64", 0.4, 12)):
        x, z, ph, ms = rh_ten_day_run(stc, x0, z0, a, dt, Om, steps, prec, th, d, log=log)
        runs[tag] = report(tag, x, z, ph, ms, x0, z0, a)
        finals[tag] = (x, z)
    x6, f6 = S.icosahedral_grid(6, return_faces=True)
    a6 = S.node_patch_areas(x6, f6)
    z6 = S.rossby_haurwitz(x6, 4)
    x, z, ph, ms = rh_ten_day_run(stc, x6, z6, a6, dt, Om, steps, "fp64", 0.7, 8, log=log)
    runs["fp64_level6_N40962"] = report("fp64 level 6", x, z, ph, ms, x6, z6, a6)
    (x64, z64), (x32, z32) = finals["fp64"], finals["fp32"]
    fp32_vs_fp64 = dict(max_position_diff=float(f"{np.abs(x32 - x64).max():.3e}"),
                        vorticity_rel_l2_diff=float(f"{metrics.rel_l2_scalar(z32, z64, a):.3e}"),
                        phase_diff_deg=round(runs["fp32"]["phase_deg"] - runs["fp64"]["phase_deg"], 5))
    r = runs["fp32"]
    result = dict(
        metric="RK4 steps of the ten-day Rossby-Haurwitz run at N=163842 (4 velocity evaluations per step)",
        value=round(1e3 / r["ms_per_rk4_step"], 2), unit="RK4 steps/s", n_gpus=1, steps=steps, warmup=0,
        ms_per_step=r["ms_per_rk4_step"], higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
        data="synthetic",
        config=dict(workload="rh4_l7 ten days (Rossby-Haurwitz n=4, icosahedral level 7, node-patch areas)", N=n,
                    theta=0.7, degree=8, n_crit=64, dt_seconds=dt, steps=steps, omega=Om,
                    closed_form_phase_deg=round(expected, 4), runs=runs, fp32_vs_fp64=fp32_vs_fp64),
    )
    print(json.dumps(result), flush=True)


AMR = dict(level0=5, eps1=0.0025, eps2=0.2, dt=0.01, days=3.0, max_levels=3, theta=0.7, degree=6, n_crit=64)


def amr_run(stc, theta, degree, log=None):
    """The Gaussian vortex of Sec. 4.3 with adaptive refinement: initial mesh
    of 10242 particles, the initial field resolved by passes that re-evaluate
    it at the live particles, then RK4 steps of dt = 0.01 day, each followed
    by one adaptation pass, for 3 days.  Returns timings, particle counts and
    the vortex track (position of the largest vorticity, daily)."""
    import torch
    import synthetic as S
    P = AMR
    x0, f0 = S.icosahedral_grid(P["level0"], return_faces=True)
    a0 = S.node_patch_areas(x0, f0)
    om = S.OMEGA_EARTH_DAY
    mesh = stc.AdaptiveMesh(x0, f0, eps1=P["eps1"], eps2=P["eps2"], omega=om, max_levels=P["max_levels"])
    mesh.set_state(torch.from_numpy(x0).cuda(), torch.from_numpy(S.gaussian_vortex_paper(x0, a0)).cuda())
    for _ in range(P["max_levels"] + 1):
        mesh.adapt()
        x, z, a = mesh.particles()
        xh, ah = x.cpu().numpy(), a.cpu().numpy()
        mesh.set_state(x.clone(), torch.from_numpy(S.gaussian_vortex_paper(xh, ah)).cuda())
    n_initial = mesh.stats()["particles"]
    ctx = stc.Context(mesh.capacity, theta=theta, degree=degree, n_crit=P["n_crit"], precision="fp64",
                      denominator="dist2")
    steps = int(round(P["days"] / P["dt"]))
    per_day = int(round(1.0 / P["dt"]))
    track, counts = [], [n_initial]

    def vortex_centre():
        x, z, _ = mesh.particles()
        k = int(torch.argmax(z).item())
        c = x[k].cpu().numpy()
        return [round(float(np.degrees(np.arcsin(c[2]))), 3), round(float(np.degrees(np.arctan2(c[1], c[0]))), 3)]

    track.append(vortex_centre())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for day in range(0, steps, per_day):
        mesh.rk4(ctx, P["dt"], om, min(per_day, steps - day))
        counts.append(mesh.stats()["particles"])
        track.append(vortex_centre())
        if log:
            log(f"  theta={theta} d={degree}: day {len(counts) - 1}, {counts[-1]} particles")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    x, z, a = mesh.particles()
    circ = float((z * a).sum().item())
    circ_abs = float((z.abs() * a).sum().item())
    ctx.close()
    mesh.close()
    return dict(seconds=round(wall, 3), ms_per_step=round(wall * 1e3 / steps, 4), steps=steps,
                particles_initial=n_initial, particles_daily=counts, vortex_track_lat_lon_deg=track,
                circulation_rel=float(f"{abs(circ) / circ_abs:.3e}"))


def bench_amr(args):
    """Adaptive refinement with time stepping: the Gaussian-vortex run of
    Sec. 4.3 (10242 initial particles, eps1 = 0.0025, eps2 = 0.2, 3 days of
    RK4 with dt = 0.01 day and one adaptation pass per step, theta 0.7, d 6,
    FP64), beside a reference run with a tighter tree (theta 0.4, d 10) whose
    vortex track it should follow."""
    from paper_2401_07361_amd import stc
    log("amr: Gaussian vortex, theta 0.7, d 6")
    r = amr_run(stc, AMR["theta"], AMR["degree"], log=log)
    log("amr: reference tree theta 0.4, d 10")
    ref = amr_run(stc, 0.4, 10, log=log)
    tr, tf = np.radians(np.array(r["vortex_track_lat_lon_deg"])), np.radians(np.array(ref["vortex_track_lat_lon_deg"]))

    def unit(ll):
        return np.stack([np.cos(ll[:, 0]) * np.cos(ll[:, 1]), np.cos(ll[:, 0]) * np.sin(ll[:, 1]), np.sin(ll[:, 0])], 1)

    sep = np.degrees(np.arccos(np.clip((unit(tr) * unit(tf)).sum(1), -1.0, 1.0)))
    result = dict(
        metric="RK4 steps with adaptive refinement per second, Gaussian vortex (10242 initial particles, 3 days)",
        value=round(r["steps"] / r["seconds"], 2), unit="RK4+AMR steps/s", n_gpus=1, steps=r["steps"], warmup=0,
        ms_per_step=r["ms_per_step"], higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
        data="synthetic",
        config=dict(workload="Gaussian vortex with AMR (Sec. 4.3)", **AMR, run=r, reference_tight_tree=dict(theta=0.4, degree=10, **ref),
                    track_separation_deg=[round(float(v), 4) for v in sep]),
    )
    print(json.dumps(result), flush=True)


def bench_ssw(args):
    """Forced RK4 of the polar-vortex collapse (Sec. 4.4) at the paper's setting
    (N = 163842, d = 6, theta = 0.7, wavenumber-1 forcing); the accuracy check
    is one evaluation at full forcing (day 8) against the FP64 direct sum of
    the forced field on 4096 seeded targets."""
    import torch
    import synthetic as S
    from paper_2401_07361_amd import stc
    from oracle import metrics

    wl = S.make_workload("ssw_l7")
    x, z, a, sub = wl["x"], wl["zeta"], wl["area"], wl["subset"]
    n = len(x)
    dt, Om, fc = wl["dt"], wl["omega"], wl["forcing"]
    fargs = (fc["k"], Om, fc["lat1"], fc["t_ramp"], fc["t_total"])
    t_check = 8.0
    xd, zd, ad = (torch.from_numpy(v).cuda() for v in (x, z, a))
    zf = zd - stc.forcing_field(xd, *fargs, t_check)
    ud = stc.direct(xd, zf, ad, targets=torch.from_numpy(sub).cuda(), denominator="dist2").cpu().numpy()
    log(f"workload ssw_l7 N={n} theta={wl['theta']} d={wl['degree']} k={fc['k']} dt={dt} days")
    runs = {}
    for prec in ("fp32", "fp64"):
        ctx = stc.Context(n, theta=wl["theta"], degree=wl["degree"], n_crit=64, precision=prec, denominator="dist2")
        ctx.set_forcing(*fargs, time=t_check)
        u = ctx.velocity(xd, zd, ad)
        shape = ctx.autotune(repeats=5)  # launch shape for this size, used by the evaluations below
        log(f"{prec}: autotuned launch shape {shape}")
        err = metrics.rel_l2_velocity(u.cpu().numpy()[sub], ud, a[sub])
        ms_eval, kern_ms_t, ph = _timed(ctx, lambda: ctx.velocity(xd, zd, ad, out=u), args.steps, args.warmup)
        cnt, ev = ctx.list_counts()
        xs, zs = xd.clone(), zd.clone()
        ctx.set_forcing(*fargs, time=0.0)
        ctx.rk4(xs, zs, ad, dt, Om, 1)   # captures the step graph
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        ctx.rk4(xs, zs, ad, dt, Om, args.steps)
        t1.record()
        torch.cuda.synchronize()
        ctx.sync()
        ms_step = t0.elapsed_time(t1) / args.steps
        t_end = ctx.forcing()[1]["time"]
        runs[prec] = dict(ms_per_rk4_step=round(ms_step, 4), ms_per_evaluation=round(ms_eval, 4), launch_shape=shape,
                          rel_l2_err_vs_fp64_direct=float(f"{err:.3e}"), phase_ms=ph, forcing_time_after=t_end,
                          near=(ev, kern_ms_t))
        log(f"{prec}: {ms_step:.3f} ms per forced RK4 step (graph), {ms_eval:.3f} ms per evaluation, E = {err:.3e}")
        ctx.close()
    r = runs["fp32"]
    roof_evals, roof_ms = r.pop("near")
    runs["fp64"].pop("near")
    result = dict(
        metric="particle velocity evals/s in forced RK4 time stepping at N=163842 (polar-vortex collapse, "
               "4 evaluations per step, one HIP graph per step)",
        value=4 * n / (r["ms_per_rk4_step"] / 1e3), unit="velocity evals/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=r["ms_per_rk4_step"], higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f32", data="synthetic",
        config=dict(workload="ssw_l7 (polar vortex, wavenumber-1 forcing, icosahedral level 7, node-patch areas)",
                    N=n, theta=wl["theta"], degree=wl["degree"], n_crit=64, dt_days=dt, omega_per_day=Om,
                    forcing=fc, error_check_day=t_check, runs=runs),
        roofline=roofline(roof_evals, roof_ms, "fp32"),
    )
    if not args.no_cpu:
        log("cpu baseline (oracle direct sum of the forced field, bounded target sample)")
        cb, _, _ = cpu_baseline(x, zf.cpu().numpy(), a, sub, budget_s=8.0, den="dist2", what="4096 seeded targets")
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


def bench_plain(args):
    """The plain method as the paper runs it: FP64 with the 1 - x.y
    denominator, theta 0.7, d 8, on the level-5 grid (N = 10242) with the
    Rossby-Haurwitz wave n = 4; accuracy against the FP64 direct sum at every
    particle."""
    import torch
    import synthetic as S
    from paper_2401_07361_amd import stc
    from oracle import metrics

    wl = S.make_workload("rh4_l5")
    x, z, a = wl["x"], wl["zeta"], wl["area"]
    n = len(x)
    log(f"workload rh4_l5 N={n} theta={wl['theta']} d={wl['degree']} fp64 1 - x.y")
    xd, zd, ad = (torch.from_numpy(v).cuda() for v in (x, z, a))
    ud = stc.direct(xd, zd, ad).cpu().numpy()
    ctx = stc.Context(n, theta=wl["theta"], degree=wl["degree"], n_crit=64, precision="fp64", denominator="dot")
    u = ctx.velocity(xd, zd, ad)
    err = metrics.rel_l2_velocity(u.cpu().numpy(), ud, a)
    ms, kern_ms, ph = _timed(ctx, lambda: ctx.velocity(xd, zd, ad, out=u), args.steps, args.warmup)
    cnt, ev = ctx.list_counts()
    ug = u.cpu().numpy()
    ctx_level = ctx.max_level
    ctx.close()
    log(f"{ms:.3f} ms per evaluation, E = {err:.3e} vs the FP64 direct sum (all {n} particles)")
    result = dict(
        metric="particle velocity evals/s at N=10242 (plain FP64 method, theta 0.7, d 8)",
        value=n / (ms / 1e3), unit="velocity evals/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(ms, 4), higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f64",
        data="synthetic",
        config=dict(workload="rh4_l5 (Rossby-Haurwitz n=4, icosahedral level 5, A = 4 pi / N)", N=n,
                    theta=wl["theta"], degree=wl["degree"], n_crit=64, precision="fp64", denominator="dot",
                    rel_l2_err_vs_fp64_direct=float(f"{err:.3e}"), lists=cnt, phase_ms=ph),
        roofline=roofline(ev, kern_ms, "fp64"),
    )
    if not args.no_cpu:
        log("cpu baseline (oracle direct sum, bounded target sample)")
        cb, _, _ = cpu_baseline(x, z, a, np.arange(n), budget_s=8.0, den="dot", what="all particles")
        # the oracle's tree code (one process) on the same input and setting
        from oracle import tree as otree
        t0 = time.perf_counter()
        ut = otree.velocity(x, z, a, theta=wl["theta"], degree=wl["degree"], n_crit=64, max_level=int(ctx_level))
        dt_tree = time.perf_counter() - t0
        cb["oracle_tree"] = dict(value=n / dt_tree, unit="velocity evals/s", cores=1, seconds=round(dt_tree, 2),
                                 max_rel_diff_gpu_vs_oracle_tree=float(f"{np.abs(ug - ut).max() / np.abs(ut).max():.3e}"))
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


LOG_FLOPS = 12  # per stream-function evaluation: 3 sub, |d|^2 5, x1/2 1, log 1 (counted as one), q*log + add 2


def bench_stream(args):
    """The stream function (Sec. 2; the logarithmic kernel through the same
    tree) on the headline workload and setting (N = 655362 Gaussian vortex,
    FP32 form, theta 0.8, d 10), checked against the FP64 direct stream
    function on the 4096 seeded targets."""
    import torch
    import synthetic as S
    from paper_2401_07361_amd import stc
    from oracle import metrics

    wl = S.make_workload("gv_l8", level=args.level)
    x, z, a, sub = wl["x"], wl["zeta"], wl["area"], wl["subset"]
    n = len(x)
    log(f"workload gv_l8 stream function N={n} theta={args.theta} d={args.degree} {args.precision}")
    xd, zd, ad = (torch.from_numpy(v).cuda() for v in (x, z, a))
    ref = stc.direct_stream(xd, zd, ad, targets=torch.from_numpy(sub).cuda(), denominator="dist2").cpu().numpy()
    ctx = stc.Context(n, theta=args.theta, degree=args.degree, n_crit=args.n_crit, precision=args.precision,
                      denominator="dist2")
    psi = ctx.stream_function(xd, zd, ad)
    err = metrics.rel_l2_scalar(psi.cpu().numpy()[sub], ref, a[sub])
    ms, kern_ms, ph = _timed(ctx, lambda: ctx.stream_function(xd, zd, ad, out=psi), args.steps, args.warmup)
    cnt, ev = ctx.list_counts()
    log(f"{ms:.3f} ms per stream-function evaluation, E = {err:.3e} vs the FP64 direct sum (4096 targets)")
    ctx.close()
    near = roofline(ev, kern_ms, args.precision, flops=LOG_FLOPS)
    result = dict(
        metric="particle stream-function evals/s at N=655362 (logarithmic kernel through the tree)",
        value=n / (ms / 1e3), unit="stream-function evals/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(ms, 4), higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32" if args.precision == "fp32" else "f64", data="synthetic",
        config=dict(workload="gv_l8 (Gaussian vortex, icosahedral level 8), stream function", N=n, theta=args.theta,
                    degree=args.degree, n_crit=args.n_crit, precision=args.precision, denominator="dist2",
                    rel_l2_err_vs_fp64_direct=float(f"{err:.3e}"), lists=cnt, phase_ms=ph),
        roofline=near,
    )
    if not args.no_cpu:
        log("cpu baseline (oracle direct stream function, bounded target sample)")
        cb, _, _ = cpu_baseline(x, z, a, sub, budget_s=10.0, den="dist2", stream=True)
        cb["unit"] = "stream-function evals/s"
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--theta", type=float, default=BENCH_THETA)
    ap.add_argument("--degree", type=int, default=BENCH_DEGREE)
    ap.add_argument("--n-crit", type=int, default=BENCH_N_CRIT)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--level", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workload", default="gv_l8",
                    choices=["gv_l8", "ensemble", "learned", "rk4", "rh10d", "amr", "ssw", "stream", "plain"])
    ap.add_argument("--autotune", action="store_true",
                    help="gv_l8: pick the interaction kernels' launch shape with the library's autotuner first")
    ap.add_argument("--copy-check", action="store_true",
                    help="also run one plain 256 MiB device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.workload == "ensemble":
        bench_ensemble(args)
        return
    if args.workload == "learned":
        bench_learned(args)
        return
    if args.workload == "rk4":
        bench_rk4(args)
        return
    if args.workload == "ssw":
        bench_ssw(args)
        return
    if args.workload == "rh10d":
        bench_rh10d(args)
        return
    if args.workload == "amr":
        bench_amr(args)
        return
    if args.workload == "stream":
        bench_stream(args)
        return
    if args.workload == "plain":
        bench_plain(args)
        return

    import torch
    import synthetic as S
    from paper_2401_07361_amd import stc

    wl = S.make_workload("gv_l8", level=args.level)
    x, z, a, subset = wl["x"], wl["zeta"], wl["area"], wl["subset"]
    n = len(x)
    log(f"workload gv_l8 N={n} theta={args.theta} d={args.degree} n_crit={args.n_crit} {args.precision}")
    xd = torch.from_numpy(x).cuda()
    zd = torch.from_numpy(z).cuda()
    ad = torch.from_numpy(a).cuda()
    sd = torch.from_numpy(subset).cuda()
    out = torch.empty((n, 3), dtype=torch.float64, device="cuda")
    den = "dist2" if args.precision == "fp32" else "dot"
    ctx = stc.Context(n, theta=args.theta, degree=args.degree, n_crit=args.n_crit,
                      precision=args.precision, denominator=den)
    if args.copy_check:
        src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        ctx.velocity(xd, zd, ad, out=out)
    ctx.sync()
    if args.autotune:
        log(f"autotuned launch shape {ctx.autotune(repeats=5)}")
    log("warmup done")

    ms, kern_ms, phase_ms = _timed(ctx, lambda: ctx.velocity(xd, zd, ad, out=out), args.steps, 0)
    log(f"timed {args.steps} steps: {ms:.3f} ms/step; k_near {kern_ms['near']:.4f} ms, k_far_targets "
        f"{kern_ms['far_targets']:.4f} ms; phases {json.dumps(phase_ms)}")

    counts, evals = ctx.list_counts()
    # accuracy: FP64 direct sum on the GPU (parity-tested against the oracle) at the 4096 targets
    scratch = stc.workspace_tensor(stc.direct_scratch_bytes(n, len(subset)))
    ud_t = stc.direct(xd, zd, ad, targets=sd, scratch=scratch)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    stc.direct(xd, zd, ad, targets=sd, out=ud_t, scratch=scratch)
    e1.record()
    torch.cuda.synchronize()
    direct_ms = e0.elapsed_time(e1)
    ud = ud_t.cpu().numpy()
    direct_evals = len(subset) * (n - 1)
    direct_tf = direct_evals * FP64_FLOPS / (direct_ms / 1e3) / 1e12
    ut = out.cpu().numpy()[subset]
    from oracle import metrics
    err = metrics.rel_l2_velocity(ut, ud, a[subset])
    log(f"E vs FP64 direct (4096 targets) = {err:.3e}; lists {counts}")

    config_tag = f"gv_l8 L{args.level} theta={args.theta} d={args.degree} n_crit={args.n_crit} {args.precision}"
    roof = roofline(evals, kern_ms, args.precision, config_tag=config_tag)

    result = dict(
        metric="particle velocity evals/s at N=655362, rel-L2 err <=1e-6 vs FP64 direct sum",
        value=n / (ms / 1e3), unit="velocity evals/s", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=round(ms, 4), higher_is_better=True, scaling="weak", vs_baseline=None,
        dtype="f32" if args.precision == "fp32" else "f64", data="synthetic",
        config=dict(workload="gv_l8 (Gaussian vortex, icosahedral level %d)" % args.level, N=n,
                    theta=args.theta, degree=args.degree, n_crit=args.n_crit, max_level=ctx.max_level,
                    precision=args.precision, denominator=den, rel_l2_err_vs_fp64_direct=float(f"{err:.3e}"),
                    err_ok=bool(err <= 1e-6), lists=counts,
                    kernel_evals=int(sum(evals.values())), phase_ms={p: round(v, 4) for p, v in phase_ms.items()},
                    kernel_source_hash=kernel_source_hash(),
                    direct_sum=dict(kernel="k_direct FP64 (1 - x.y), 4096 targets x all sources", ms=round(direct_ms, 4),
                                    evals_per_s=direct_evals / (direct_ms / 1e3), tflops=round(direct_tf, 3),
                                    frac_of_fp64_peak=round(direct_tf / PEAK_FP64_TFLOPS, 4))),
        roofline=roof,
    )
    ctx.close()
    if not args.no_cpu:
        log("cpu baseline (oracle direct sum on a bounded target sample)")
        cb, sample, uo = cpu_baseline(x, z, a, subset)
        pos = np.searchsorted(subset, sample)
        cb["rel_l2_err_gpu_vs_oracle_on_sample"] = float(f"{metrics.rel_l2_velocity(ut[pos], uo, a[sample]):.3e}")
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
