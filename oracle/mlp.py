"""O5a: the learned form's network in plain NumPy.  TEST INFRASTRUCTURE ONLY.

The network: 12 inputs -> 64 -> 64 -> 4 outputs with ReLU hidden layers.
Parameters are one flat vector of 5252 values: W1 [12][64] (input f to hidden
h), b1 [64], W2 [64][64], b2 [64], W3 [64][4], b3 [4].  Outputs: o0 the
acceptance logit, o1..o3 ordinal logits (degree above 4, 6, 8).  Loss per
row, averaged over the batch:
    a(y0) BCE(o0, y0) + y0 * sum_{k=1..3} h(y_k) BCE(o_k, y_k),
BCE(o, y) = max(o, 0) - o y + log(1 + exp(-|o|)) (logits), so the ordinal
targets count only where the pair is acceptable.  The two costly mistakes,
accepting a pair labelled reject and choosing a degree below the labelled
one, weigh W_REJECT and W_HIGHER times the others: a(0) = W_REJECT,
a(1) = 1, h(1) = W_HIGHER, h(0) = 1.  A constant network's best logits then
sit ln W lower (acceptance) and higher (ordinals) than the labels' log-odds,
so the trained network's own decisions lean to the safe side and the bias
shifts of the calibration after training stay small.

Everything is FP64.  `act_round`, when given, is applied to the hidden
activations and to the back-propagated pre-activation gradients, the places
where the GPU kernels round to BF16 before a matrix product; it lets a test
compare against the kernels' own precision (decisions that depend on a
rounded value are taken in the precision of the kernel).
"""

import numpy as np

N_IN, N_H, N_OUT = 12, 64, 4
SLICES = {
    "W1": (0, (12, 64)), "b1": (768, (64,)), "W2": (832, (64, 64)),
    "b2": (4928, (64,)), "W3": (4992, (64, 4)), "b3": (5248, (4,)),
}
N_PARAMS = 5252


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    return {k: theta[o:o + int(np.prod(s))].reshape(s) for k, (o, s) in SLICES.items()}


def pack(p):
    out = np.zeros(N_PARAMS)
    for k, (o, s) in SLICES.items():
        out[o:o + int(np.prod(s))] = np.asarray(p[k], dtype=np.float64).ravel()
    return out


def bf16_round(a):
    """Round float values to BF16 (round to nearest, ties to even) and back."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def bf16_bits(a):
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def from_bf16_bits(b):
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def forward(theta, x, act_round=None):
    """x (n, 12 or 16) -> outputs (n, 4) and the intermediate values."""
    p = unpack(theta)
    x = np.asarray(x, dtype=np.float64)[:, :N_IN]
    r = act_round if act_round is not None else (lambda v: v)
    z1 = x @ p["W1"] + p["b1"]
    h1 = r(np.maximum(z1, 0.0))
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = r(np.maximum(z2, 0.0))
    o = h2 @ p["W3"] + p["b3"]
    return o, dict(x=x, z1=z1, h1=h1, z2=z2, h2=h2)


W_REJECT = 8.0
W_HIGHER = 8.0


def bce(o, y):
    return np.maximum(o, 0.0) - o * y + np.log1p(np.exp(-np.abs(o)))


def _weights(y):
    """Per-row weight of the acceptance term and per-row, per-ordinal weights."""
    return 1.0 + (W_REJECT - 1.0) * (1.0 - y[:, 0]), 1.0 + (W_HIGHER - 1.0) * y[:, 1:]


def loss(theta, x, y, act_round=None):
    o, _ = forward(theta, x, act_round)
    y = np.asarray(y, dtype=np.float64)
    wa, wo = _weights(y)
    per = wa * bce(o[:, 0], y[:, 0]) + y[:, 0] * (wo * bce(o[:, 1:], y[:, 1:])).sum(1)
    return float(per.mean())


def _sigmoid(o):
    return 0.5 * (1.0 + np.tanh(0.5 * o))


def grad(theta, x, y, act_round=None):
    """Gradient of `loss` with respect to the flat parameters (chain rule
    written out layer by layer)."""
    p = unpack(theta)
    o, c = forward(theta, x, act_round)
    y = np.asarray(y, dtype=np.float64)
    n = len(o)
    r = act_round if act_round is not None else (lambda v: v)
    wa, wo = _weights(y)
    d3 = np.empty_like(o)
    d3[:, 0] = wa * (_sigmoid(o[:, 0]) - y[:, 0]) / n
    d3[:, 1:] = y[:, :1] * wo * (_sigmoid(o[:, 1:]) - y[:, 1:]) / n
    d3r = r(d3)
    g = {"W3": c["h2"].T @ d3r, "b3": d3.sum(0)}
    d2 = (d3r @ p["W3"].T) * (c["z2"] > 0)
    d2r = r(d2)
    g["W2"] = c["h1"].T @ d2r
    g["b2"] = d2.sum(0)
    d1 = (d2r @ p["W2"].T) * (c["z1"] > 0)
    d1r = r(d1)
    g["W1"] = c["x"].T @ d1r
    g["b1"] = d1.sum(0)
    return pack(g)


def decide(outputs):
    """(accept, degree class) from network outputs: accept iff o0 > 0; class
    = number of positive ordinal logits."""
    o = np.asarray(outputs)
    return o[:, 0] > 0, (o[:, 1:] > 0).sum(1)


def calibration_grid():
    """The bias shifts a calibration tries, in increasing order: 0, then 200
    values in geometric progression from 1e-3 to 64."""
    g = np.zeros(201)
    g[1:] = 1e-3 * (64.0 / 1e-3) ** (np.arange(200) / 199.0)
    g[-1] = 64.0
    return g


def calibration_shifts(outputs, labels, max_false_accept, max_under_class):
    """(da, dc): the smallest grid values at which (a) at most
    max_false_accept of all samples are labelled reject (y0 = 0) but accepted
    with the acceptance logit lowered by da (o0 - da > 0), and (b) at most
    max_under_class of the samples labelled accept and still accepted get
    fewer positive ordinal logits, raised by dc, than their label asks for
    (y1 + y2 + y3).  The largest grid value when no value meets a bar; 0 when
    there is nothing to count.  Plain loops over the grid."""
    o = np.asarray(outputs, dtype=np.float64)
    y = np.asarray(labels, dtype=np.float64)
    grid = calibration_grid()
    n = len(o)
    if n == 0:
        return 0.0, 0.0
    acc = y[:, 0] > 0
    da = grid[-1]
    for d in grid:
        if np.count_nonzero((o[:, 0] - d > 0) & ~acc) / n <= max_false_accept:
            da = d
            break
    keep = acc & (o[:, 0] - da > 0)
    if not keep.any():
        return float(da), 0.0
    need = np.rint(y[keep, 1:].sum(1))
    dc = grid[-1]
    for d in grid:
        under = (o[keep, 1:] + d > 0).sum(1) < need
        if np.count_nonzero(under) / keep.sum() <= max_under_class:
            dc = d
            break
    return float(da), float(dc)


def apply_shifts(param_bits, da, dc):
    """BF16 parameter bits with b3[0] lowered by da and b3[1..3] raised by dc
    (the shift in FP64, rounded to FP32 and then to BF16)."""
    p = from_bf16_bits(param_bits)
    o = SLICES["b3"][0]
    p[o] -= da
    p[o + 1:o + 4] += dc
    out = np.asarray(param_bits, dtype=np.uint16).copy()
    out[o:o + 4] = bf16_bits(p[o:o + 4])
    return out


def init_params(seed):
    """He-style random initialisation (used as a starting point in tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {"W1": rng.standard_normal((12, 64)) * np.sqrt(2.0 / 12), "b1": np.zeros(64),
         "W2": rng.standard_normal((64, 64)) * np.sqrt(2.0 / 64), "b2": np.zeros(64),
         "W3": rng.standard_normal((64, 4)) * np.sqrt(2.0 / 64), "b3": np.zeros(4)}
    return pack(p)
