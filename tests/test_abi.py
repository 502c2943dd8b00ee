"""The C ABI library loads, exports every declared symbol, and validates scalar
arguments on the host (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gp2s.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gp2s_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    import paper_2512_06143_amd.gp2s as B
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(B.lib, n), n
    assert set(names) == set(B.EXPORTED)
    assert B.lib.gp2s_abi_version() == 2


def _ctx():
    import paper_2512_06143_amd.gp2s as B
    ctx = ctypes.c_void_p()
    assert B.lib.gp2s_create(ctypes.byref(ctx), None, B.ALLOC_FN(), B.FREE_FN(), None) == 0
    return B, ctx


def _params(B, **kw):
    import numpy as np
    d = dict(dim=2, radius=0.05, bump_width=0.6, noise_var=1e-4, centers=np.array([[0.5, 0.5]]),
             weights=np.array([1.0]))
    d.update(kw)
    return B.HostParams(**d).to_c()


@pytest.mark.parametrize("kw,n,code", [
    (dict(), 10, 0),
    (dict(dim=4, centers=[[0.5] * 4]), 10, 1),
    (dict(radius=0.0), 10, 1),
    (dict(radius=float("nan")), 10, 7),
    (dict(bump_width=-1.0), 10, 1),
    (dict(noise_var=-1e-3), 10, 1),
    (dict(weights=[float("inf")]), 10, 7),
    (dict(), 0, 1),
    (dict(), 1 << 31, 1),
    (dict(kernel=1), 10, 0),
    (dict(kernel="c6"), 10, 0),
    (dict(kernel=2), 10, 1),
    (dict(radii=[0.05, 0.02]), 10, 0),
    (dict(radii=[0.05, 0.0]), 10, 1),
    (dict(radii=[0.05, float("nan")]), 10, 7),
    (dict(ls_weights=[0.7]), 10, 0),
    (dict(ls_weights=[25.0]), 10, 1),
    (dict(ls_weights=[float("inf")]), 10, 7),
    (dict(ff_groups=[0]), 10, 0),
    (dict(ff_groups=[16]), 10, 1),
    (dict(ff_groups=[0], radii=[0.05, 0.05]), 10, 1),
])
def test_host_validation(kw, n, code):
    B, ctx = _ctx()
    p, keep = _params(B, **kw)
    assert B.lib.gp2s_check_params(ctx, n, ctypes.byref(p)) == code
    if code:
        assert B.lib.gp2s_last_error(ctx)
    B.lib.gp2s_destroy(ctx)


def test_entry_points_reject_bad_arguments_without_gpu():
    B, ctx = _ctx()
    p, keep = _params(B)
    h = ctypes.c_void_p()
    o0 = B.default_opts()
    rep = B.PredictReport()
    assert B.lib.gp2s_predict(ctx, None, 4, 1234, 1234, ctypes.byref(o0), 1234, None, ctypes.byref(rep)) == 1
    # invalid precision / null pointers are rejected before any device call
    assert B.lib.gp2s_assemble(ctx, 10, None, ctypes.byref(p), 0, ctypes.byref(h)) == 1
    assert B.lib.gp2s_assemble(ctx, 10, 1234, ctypes.byref(p), 9, ctypes.byref(h)) == 1
    o = B.default_opts()
    o.n_probes = 65
    assert B.lib.gp2s_lml(ctx, None, None, ctypes.byref(o), None, None) == 1
    assert B.lib.gp2s_spmv(ctx, None, 1, None, None) == 1
    assert B.lib.gp2s_matrix_import(ctx, 5, 3, 1, 1, 1, 0, ctypes.byref(h)) == 1  # nnz < n
    assert B.lib.gp2s_create(None, None, B.ALLOC_FN(), B.FREE_FN(), None) == 1
    assert B.lib.gp2s_status_string(6) == b"iteration did not converge"
    B.lib.gp2s_destroy(ctx)


def test_timing_mask_host_side():
    """The timing switches need no device while nothing is pending: a null context is
    rejected, and a set mask leaves every total at zero."""
    B, ctx = _ctx()
    assert B.lib.gp2s_set_timing_mask(None, 1) == 1
    assert B.lib.gp2s_set_timing_mask(ctx, (1 << B.NUM_TIMERS) - 1) == 0
    st = B.Stats()
    assert B.lib.gp2s_get_stats(ctx, ctypes.byref(st)) == 0
    assert all(c == 0 for c in st.count) and all(t == 0.0 for t in st.ms)
    assert B.lib.gp2s_set_timing(ctx, 0) == 0
    assert B.lib.gp2s_get_stats(None, ctypes.byref(st)) == 1
    B.lib.gp2s_destroy(ctx)


def test_default_opts():
    import paper_2512_06143_amd.gp2s as B
    o = B.default_opts()
    assert (o.n_probes, o.max_iter, o.tol) == (64, 20000, 1e-8)
