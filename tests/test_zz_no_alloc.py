"""GPU: stc_direct_noalloc (the direct sum whose chunk partial sums live in
the library's static device scratch array) against stc_direct on the same
inputs, through the C ABI.

Both entry points split the sources into the same chunks and reduce them in
the same fixed order, so the outputs are compared bitwise.  Two calls in a
row on the same GPU, the second smaller, check that the shared array's
contents from the first call do not leak into the second.
"""

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def sphere_points(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 3))
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def make_case(n, m, seed):
    rng = np.random.default_rng(seed + 1000)
    x = sphere_points(n, seed)
    z = rng.uniform(-1.0, 1.0, n)
    a = np.full(n, 4.0 * np.pi / n)
    t = np.sort(rng.choice(n, size=m, replace=False)).astype(np.int64)
    return [torch.from_numpy(v).cuda() for v in (x, z, a, t)]


# (n, m) of the first and the second (smaller) call; each splits the sources
CASES = [
    ((655362, 4096), (163842, 1000)),
    ((40962, 4096), (10242, 100)),
]


@pytest.mark.parametrize("precision,den", [("fp64", "dot"), ("fp64", "dist2"), ("fp32", "dist2")])
@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_direct_matches_direct_twice(stc_lib, precision, den, first, second):
    stc = stc_lib
    for k, (n, m) in enumerate((first, second)):
        say(f"noalloc direct: call {k + 1} n={n} m={m} {precision} {den}")
        x, z, a, t = make_case(n, m, seed=7 + k)
        ref = stc.direct(x, z, a, targets=t, precision=precision, denominator=den)
        out = torch.full((m, 3), float("nan"), dtype=torch.float64, device="cuda")
        stc.direct_noalloc(x, z, a, targets=t, precision=precision, denominator=den, out=out)
        r, o = ref.cpu().numpy(), out.cpu().numpy()
        assert np.isfinite(o).all()
        assert np.array_equal(r, o), f"max diff {np.abs(r - o).max():.3e}"
