"""CPU-only checks of the HIP library: it loads, exports every function the
header declares, and its host-side geometry and interpolation tables agree
with the oracle's independent implementation.  No device work is done."""

import ctypes
import os
import re

import numpy as np
import pytest

from oracle import geometry as G
from oracle import interp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stc.h")


@pytest.fixture(scope="module")
def stc():
    from paper_2401_07361_amd import stc as mod
    return mod


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stc_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_function(stc):
    lib = stc.library()
    names = _declared_functions()
    assert len(names) >= 25
    for name in names:
        assert hasattr(lib, name), name


def test_geometry_tables_bitwise_equal_to_oracle(stc):
    L = 4
    v, c, r = stc.geometry_tables(L)
    geom = G.TreeGeometry(L)
    for lvl in range(L + 1):
        off = G.level_offset(lvl)
        nl = 20 * 4 ** lvl
        np.testing.assert_array_equal(v[off:off + nl], geom.verts[lvl])
        np.testing.assert_array_equal(c[off:off + nl], geom.center[lvl])
        np.testing.assert_array_equal(r[off:off + nl], geom.radius[lvl])


@pytest.mark.parametrize("d", [1, 2, 5, 8, 10, 12, 14])
def test_reference_tables_match_oracle_points(stc, d):
    pts, vinv = stc.reference_tables(d)
    np.testing.assert_allclose(pts, interp.reference_points(d), atol=2e-15)
    V = interp.basis(interp.reference_points(d), d)   # V[m, k] = B_k(b_m)
    # vinv[k, m] = (V^{-1})_{km}
    np.testing.assert_allclose(vinv @ V, np.eye(len(pts)), atol=1e-9)
    np.testing.assert_allclose(V @ vinv, np.eye(len(pts)), atol=1e-9)


def test_sizes_and_defaults(stc):
    assert [stc.n_basis(d) for d in (2, 4, 6, 8, 10, 12, 14)] == [6, 15, 28, 45, 66, 91, 120]
    assert stc.n_basis(0) == 0 and stc.n_basis(15) == 0
    assert stc.total_nodes(0) == 20 and stc.total_nodes(7) == 436900
    from oracle.tree import default_max_level
    for n in (12, 642, 10242, 163842, 655362, 2621442):
        for nc in (16, 64):
            assert stc.default_max_level(n, nc) == default_max_level(n, nc)


def test_invalid_arguments_are_rejected_without_device_work(stc):
    lib = stc.library()
    p = stc.Params()
    lib.stc_default_params(ctypes.byref(p))
    ctx = ctypes.c_void_p()
    bad = [("theta", 0.0), ("theta", 1.5), ("degree", 0), ("degree", 15), ("n_crit", 0),
           ("max_level", 13), ("precision", 7), ("denominator", 3)]
    for field, val in bad:
        q = stc.Params()
        ctypes.memmove(ctypes.byref(q), ctypes.byref(p), ctypes.sizeof(p))
        setattr(q, field, val)
        nb = ctypes.c_size_t(0)
        assert lib.stc_workspace_size(ctypes.byref(q), 1000, ctypes.byref(nb)) == 1, field
        assert lib.stc_create(ctypes.byref(q), 1000, None, 0, None, ctypes.byref(ctx)) == 1, field
    # FP32 is only offered with the |x-y|^2/2 denominator
    q = stc.Params()
    ctypes.memmove(ctypes.byref(q), ctypes.byref(p), ctypes.sizeof(p))
    q.precision = 1
    assert lib.stc_create(ctypes.byref(q), 1000, None, 0, None, ctypes.byref(ctx)) == 1
    assert lib.stc_create(ctypes.byref(p), -1, None, 0, None, ctypes.byref(ctx)) == 1
    # NULL context and NULL pointers
    assert lib.stc_tree_build(None, 10, None) == 1
    assert lib.stc_sync(None) == 1
    assert lib.stc_direct(None, 10, None, None, None, 10, None, 0, 0, None, None, 0) == 1
    assert lib.stc_direct(None, 10, None, None, None, 5, None, 0, 0, None, None, 0) == 1   # m != n without targets
    assert lib.stc_direct(None, 0, None, None, None, 0, None, 0, 0, None, None, 0) == 0    # empty: no-op
    # vorticity forcing: invalid parameters and NULL pointers are refused on the host
    import math
    good = (1, 2 * math.pi, math.pi / 3, 4.0, 15.0, 0.0)
    assert lib.stc_set_forcing(None, None) == 1
    assert lib.stc_forcing_field(None, None, 10, None, None) == 1
    assert lib.stc_forcing_field(None, ctypes.byref(stc.Forcing(*good)), 10, None, None) == 1
    assert lib.stc_forcing_field(None, ctypes.byref(stc.Forcing(*good)), 0, None, None) == 0   # empty: no-op
    for i, v in [(0, 17), (0, -1), (2, 0.0), (2, 1.6), (3, 0.0), (4, 7.9), (1, float("nan")), (5, float("inf"))]:
        f = list(good)
        f[i] = v
        assert lib.stc_forcing_field(None, ctypes.byref(stc.Forcing(*f)), 0, None, None) == 1, (i, v)
    assert lib.stc_get_forcing(None, None, None) == 1
    assert stc.status_string(2).startswith("interaction list")
    assert stc.status_string(6).startswith("workspace")
    assert stc.status_string(7).startswith("non-finite")


def test_workspace_is_sized_and_checked_on_the_host(stc):
    """The context's device buffers all come from the caller's workspace:
    its size grows with n_max and the degree, and a missing, misaligned or
    short workspace is refused (STC_ERR_WORKSPACE) before any device work."""
    lib = stc.library()
    p = stc.Params()
    lib.stc_default_params(ctypes.byref(p))
    sizes = {}
    for n in (1000, 10242, 163842):
        for d in (4, 10):
            p.degree = d
            nb = ctypes.c_size_t(0)
            assert lib.stc_workspace_size(ctypes.byref(p), n, ctypes.byref(nb)) == 0
            sizes[n, d] = nb.value
    assert sizes[1000, 4] < sizes[10242, 4] < sizes[163842, 4]
    assert all(sizes[n, 4] < sizes[n, 10] for n in (1000, 10242, 163842))
    # 8 B keys x 6 list buffers per entry at 16 entries per particle dominate
    assert sizes[163842, 10] > 6 * 8 * 16 * 163842
    nb = ctypes.c_size_t(0)
    assert lib.stc_workspace_size_batched(ctypes.byref(p), 3, 10242, 30000, ctypes.byref(nb)) == 0
    assert nb.value > sizes[10242, 10]
    p.degree = 8
    assert lib.stc_workspace_size(ctypes.byref(p), 10242, ctypes.byref(nb)) == 0
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)   # never dereferenced: the size check comes first
    assert lib.stc_create(ctypes.byref(p), 10242, None, nb.value, None, ctypes.byref(ctx)) == 6
    assert lib.stc_create(ctypes.byref(p), 10242, fake, nb.value - 1, None, ctypes.byref(ctx)) == 6
    assert lib.stc_create(ctypes.byref(p), 10242, ctypes.c_void_p((1 << 20) + 8), nb.value, None,
                          ctypes.byref(ctx)) == 6   # not 256-byte aligned
    assert not ctx.value
    sb = ctypes.c_size_t(123)
    assert lib.stc_direct_scratch_size(0, 0, 0, 0, ctypes.byref(sb)) == 0 and sb.value == 0
    assert lib.stc_direct_scratch_size(10, 10, 1, 0, ctypes.byref(sb)) == 1   # FP32 needs |x-y|^2/2
