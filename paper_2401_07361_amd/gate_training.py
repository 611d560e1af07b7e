"""Training the learned form's gating network on the GPU.

The training data are measured by the tree code itself: for each input,
stc_learned_samples takes the candidates of the wider criterion theta_max,
measures every candidate's error at the four degrees against its exact pair
sum and labels it against a tolerance (relative to stc_label_scale of the
fixed-degree velocity); stc_mlp_train then runs Adam with the library's BF16
forward and backward kernels, and stc_mlp_calibrate shifts the output biases.
This module only sequences those calls over a set of inputs (device tensors
the caller provides).
"""

import numpy as np

from . import stc


def velocity_scale(u):
    """4 pi times the root mean square speed (stc_label_scale): the size of W
    (the sum before the cross product), the unit the label tolerance is given
    in."""
    return float(stc.label_scale(u).item())


def collect(inputs, tol_rel, theta, theta_max, degree=10, n_crit=64, cap_per_input=None, log=None,
            max_samples=None):
    """Features (m, 16) BF16 and labels (m, 4) float32 from the inputs
    (an iterable of (x, zeta, area) device tensors, consumed lazily); the
    label tolerance of an input is tol_rel times its velocity scale (from a
    fixed-degree evaluation of the same context).  With max_samples, inputs
    are taken until that many samples are collected and the result is cut to
    exactly max_samples rows."""
    import torch
    feats, labs = [], []
    total = 0
    for i, (x, z, a) in enumerate(inputs):
        n = x.shape[0]
        cap = cap_per_input or 4 * n
        ctx = stc.Context(n, theta=theta, theta_max=theta_max, degree=degree, n_crit=n_crit, precision="fp64",
                          denominator="dist2", learned=True)
        u = ctx.velocity(x, z, a)            # no model: the fixed-degree method
        scale = velocity_scale(u)
        ctx.tree_build(x)
        ctx.upward(z, a)
        f, y, _, m = ctx.learned_samples(tol_rel * scale, cap)
        ctx.close()
        feats.append(f.clone())
        labs.append(y.clone())
        total += f.shape[0]
        if log:
            yn = y.cpu().numpy()
            log(f"input {i}: N={n} candidates {m} accepted {yn[:, 0].mean():.3f} "
                f"class mean {(yn[:, 1:].sum(1)[yn[:, 0] > 0]).mean():.2f} (total {total})")
        if max_samples is not None and total >= max_samples:
            break
    F, Y = torch.cat(feats), torch.cat(labs)
    if max_samples is not None:
        F, Y = F[:max_samples].contiguous(), Y[:max_samples].contiguous()
    return F, Y


def train(features, labels, epochs=8, batch=4096, lr=2e-3, seed=0, init_seed=1):
    """Trained BF16 parameters and the per-step losses."""
    import torch
    rng = np.random.Generator(np.random.PCG64(init_seed))
    p = np.zeros(stc.mlp_param_count(), dtype=np.float32)
    # He initialisation of the three weight blocks, zero biases
    p[0:768] = rng.standard_normal(768) * np.sqrt(2.0 / 12)
    p[832:4928] = rng.standard_normal(4096) * np.sqrt(2.0 / 64)
    p[4992:5248] = rng.standard_normal(256) * np.sqrt(2.0 / 64)
    master = torch.from_numpy(p).to(features.device)
    params, losses = stc.mlp_train(features, labels, master, epochs, batch, lr, seed=seed)
    return params, losses


def calibrate(features, labels, params, max_false_accept=1e-3, max_under_class=1e-3):
    """Shifts the output biases (stc_mlp_calibrate) so that, on the given
    samples, at most max_false_accept of them are accepted against their
    label and at most max_under_class of the correctly accepted ones get a
    lower degree class than labelled.  Returns new BF16 parameters and the two
    shifts."""
    newp, shifts = stc.mlp_calibrate(features, labels, params, max_false_accept, max_under_class)
    da, dc = shifts.cpu().tolist()
    return newp, float(da), float(dc)
