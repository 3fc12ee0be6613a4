"""C ABI checks that need no GPU: exported symbols and host-side validation.

No test here launches a kernel: every call either fails validation before
any HIP call, or is a T = 0 sweep, which enqueues nothing.
"""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stencil5d.h")

from paper_2001_01473_amd import _lib  # noqa: E402

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH),
                                reason="libstencil5d.so not built")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(s5d_[a-z_]+)\s*\(", text)))


def test_header_declares_binding_exports():
    assert declared_symbols() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_package_import_does_not_load_oracle():
    import sys
    import paper_2001_01473_amd  # noqa: F401
    mod = sys.modules["paper_2001_01473_amd"]
    assert "oracle" not in getattr(mod, "__dict__", {})
    src = open(os.path.join(ROOT, "paper_2001_01473_amd", "__init__.py")).read()
    src += open(os.path.join(ROOT, "paper_2001_01473_amd", "_lib.py")).read()
    assert "import oracle" not in src and "from oracle" not in src


def _create(ndim=2, radius=1, box=False, dtype=_lib.F64, accum=0, interior=(64, 64),
            steps=4, coeffs=None, tuning=None, n_coeffs=None):
    lib = _lib.load()
    if coeffs is None:
        n = (2 * radius + 1) ** ndim if box else 2 * radius * ndim + 1
        coeffs = np.full(n, 1.0 / n)
    d, keep = _lib.make_desc(ndim, radius, box, dtype, accum, interior, steps, coeffs)
    if n_coeffs is not None:
        d.n_coeffs = n_coeffs
    h = ctypes.c_void_p()
    st = lib.s5d_plan_create(ctypes.byref(d), ctypes.byref(tuning) if tuning else None,
                             ctypes.byref(h))
    return st, h


FULL = dict(bt=2, stream_chunk=32, cells_per_lane=4)


@pytest.mark.parametrize("kw,code", [
    (dict(ndim=4), _lib.S5D_EINVAL),
    (dict(ndim=1), _lib.S5D_EINVAL),
    (dict(radius=0), _lib.S5D_EINVAL),
    (dict(steps=-1), _lib.S5D_EINVAL),
    (dict(n_coeffs=4), _lib.S5D_EINVAL),
    (dict(interior=(0, 5)), _lib.S5D_EINVAL),
    (dict(dtype=7), _lib.S5D_EINVAL),
    (dict(accum=1, dtype=_lib.F64), _lib.S5D_EINVAL),
    (dict(coeffs=np.array([0.2, 0.2, np.nan, 0.2, 0.2])), _lib.S5D_EINVAL),
    (dict(radius=4, box=True), _lib.S5D_EUNSUPPORTED),  # float64 81-point box: no b_T = 2 variant fits
    (dict(radius=5), _lib.S5D_EUNSUPPORTED),
])
def test_plan_create_rejects(kw, code):
    st, h = _create(tuning=_lib.make_tuning(**FULL), **kw)
    assert st == code, (_lib.status_string(st), _lib.last_error())
    assert h.value is None
    assert _lib.last_error() != ""


def test_plan_create_rejects_bad_tuning():
    st, _ = _create(tuning=_lib.make_tuning(bt=-1))
    assert st == _lib.S5D_EINVAL
    st, _ = _create(tuning=_lib.make_tuning(tile0=100, stream_chunk=8))
    assert st == _lib.S5D_EINVAL
    st, _ = _create(tuning=_lib.make_tuning(bt=15, stream_chunk=8, cells_per_lane=4))
    assert st == _lib.S5D_EUNSUPPORTED
    bad = _lib.make_tuning(**FULL)
    bad.struct_size = 4
    st, _ = _create(tuning=bad)
    assert st == _lib.S5D_EINVAL


def test_null_arguments():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.s5d_plan_create(None, None, ctypes.byref(h)) == _lib.S5D_EINVAL
    d, keep = _lib.make_desc(2, 1, False, _lib.F64, 0, (8, 8), 1, np.full(5, 0.2))
    assert lib.s5d_plan_create(ctypes.byref(d), None, None) == _lib.S5D_EINVAL
    d.struct_size = 8
    assert lib.s5d_plan_create(ctypes.byref(d), None, ctypes.byref(h)) == _lib.S5D_EINVAL
    assert lib.s5d_plan_query(None, None, None) == _lib.S5D_EINVAL
    assert lib.s5d_run(None, None, None, None, None) == _lib.S5D_EINVAL
    lib.s5d_plan_destroy(None)


def test_plan_query_and_run_validation():
    lib = _lib.load()
    st, h = _create(interior=(100, 300), steps=7, tuning=_lib.make_tuning(**FULL))
    assert st == _lib.S5D_OK, _lib.last_error()
    t = _lib.make_tuning()
    nb = ctypes.c_int64()
    assert lib.s5d_plan_query(h, ctypes.byref(t), ctypes.byref(nb)) == _lib.S5D_OK
    assert (t.bt, t.stream_chunk, t.cells_per_lane, t.tile0) == (2, 32, 4, 256)
    assert nb.value == 102 * 302 * 8
    idx = ctypes.c_int32(-1)
    # null, overlapping and misaligned buffers are refused before any HIP call
    assert lib.s5d_run(h, None, ctypes.c_void_p(4096), None, ctypes.byref(idx)) == _lib.S5D_EINVAL
    assert lib.s5d_run(h, ctypes.c_void_p(1 << 20), ctypes.c_void_p((1 << 20) + 64), None,
                       ctypes.byref(idx)) == _lib.S5D_EINVAL
    assert lib.s5d_run(h, ctypes.c_void_p((1 << 24) + 4), ctypes.c_void_p(1 << 28), None,
                       ctypes.byref(idx)) == _lib.S5D_EINVAL
    lib.s5d_plan_destroy(h)


def test_zero_steps_enqueues_nothing():
    lib = _lib.load()
    st, h = _create(steps=0, tuning=_lib.make_tuning(**FULL))
    assert st == _lib.S5D_OK
    idx = ctypes.c_int32(-1)
    # fake, never dereferenced addresses: T = 0 makes no HIP call at all
    assert lib.s5d_run(h, ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 28), None,
                       ctypes.byref(idx)) == _lib.S5D_OK
    assert idx.value == 0
    lib.s5d_plan_destroy(h)


def test_bt_clamped_to_steps():
    lib = _lib.load()
    st, h = _create(steps=3, tuning=_lib.make_tuning(bt=8, stream_chunk=16, cells_per_lane=4))
    assert st == _lib.S5D_OK
    t = _lib.make_tuning()
    lib.s5d_plan_query(h, ctypes.byref(t), None)
    assert t.bt == 3
    lib.s5d_plan_destroy(h)


def test_status_strings():
    assert _lib.status_string(_lib.S5D_OK) == "S5D_OK"
    assert _lib.status_string(_lib.S5D_EUNSUPPORTED) == "S5D_EUNSUPPORTED"
    assert _lib.status_string(99) == "S5D_UNKNOWN"


def test_error_norms_validation():
    lib = _lib.load()
    vp = ctypes.c_void_p
    g, o, out, ws = vp(0x10000), vp(0x20000), vp(0x30000), vp(0x40000)
    need = lib.s5d_error_norms_workspace_bytes(1000)
    assert need == 40 and lib.s5d_error_norms_workspace_bytes(-1) == -1
    assert lib.s5d_error_norms_workspace_bytes(1 << 40) == 2048 * 40
    cases = [
        (g, 0, o, 1, -1, out, ws, need),          # n < 0
        (g, 2, o, 1, 1000, out, ws, need),        # bad dtype
        (g, 0, o, 1, 1000, vp(0), ws, need),      # out NULL
        (g, 0, o, 1, 1000, out, vp(0), need),     # workspace NULL
        (vp(0), 0, o, 1, 1000, out, ws, need),    # got NULL
        (vp(0x10004), 0, o, 1, 1000, out, ws, need),  # got misaligned
        (g, 0, o, 1, 1000, out, ws, need - 8),    # workspace too small
        (g, 0, o, 1, 1000, vp(0x40008), ws, need),  # out inside the workspace
    ]
    for args in cases:
        st = lib.s5d_error_norms(*args, None)
        assert st == _lib.S5D_EINVAL, args
        assert _lib.last_error()


def test_kernel_family_validation():
    st, _ = _create(tuning=_lib.make_tuning(kernel=5))
    assert st == _lib.S5D_EINVAL
    # direct kernels take no blocking parameters
    st, _ = _create(tuning=_lib.make_tuning(kernel="direct", bt=2))
    assert st == _lib.S5D_EINVAL
    # blocking asked for a stencil without a blocked variant
    st, _ = _create(ndim=3, radius=3, interior=(8, 8, 8), tuning=_lib.make_tuning(kernel="blocked"))
    assert st == _lib.S5D_EUNSUPPORTED


def test_direct_plan_needs_a_device():
    """A direct plan uploads its coefficient table at creation: without a GPU
    that is a clean S5D_EDEVICE, never a crash."""
    st, h = _create(radius=4, box=True)
    if st == _lib.S5D_OK:  # a GPU is present
        _lib.load().s5d_plan_destroy(h)
    else:
        assert st == _lib.S5D_EDEVICE, _lib.last_error()


def _create_expr(expr, ndim=2, radius=1, box=False, dtype=_lib.F64, accum=0, interior=(64, 64),
                 steps=4, coeffs=None, tuning=None):
    lib = _lib.load()
    d, keep = _lib.make_desc(ndim, radius, box, dtype, accum, interior, steps, coeffs, expr)
    h = ctypes.c_void_p()
    st = lib.s5d_plan_create(ctypes.byref(d), ctypes.byref(tuning) if tuning else None, ctypes.byref(h))
    if st == _lib.S5D_OK:
        lib.s5d_plan_destroy(h)
    return st


def test_expression_descriptor_validation():
    """Coefficient counts per expression, the gradient2d shape, the divisor,
    compensated accumulation and direct kernels (all checked on the host)."""
    E = _lib
    ok = E.S5D_OK
    assert _create_expr(E.EXPR_DIV, coeffs=[1, 2, 3, 4, 5, 15]) == ok            # j2d5pt
    assert _create_expr(E.EXPR_DIV, coeffs=[1, 2, 3, 4, 5]) == E.S5D_EINVAL      # c0 missing
    assert _create_expr(E.EXPR_DIV, coeffs=[1, 2, 3, 4, 5, 0]) == E.S5D_EINVAL   # c0 = 0
    assert _create_expr(E.EXPR_DIV, radius=2, coeffs=np.ones(10)) == ok          # j2d9pt
    assert _create_expr(E.EXPR_DIV, box=True, coeffs=np.ones(10)) == ok          # j2d9pt-gol
    assert _create_expr(E.EXPR_DIV, ndim=3, box=True, interior=(20, 30, 40), coeffs=np.ones(28)) == ok
    assert _create_expr(E.EXPR_GRADIENT, coeffs=[0.5, 1.5]) == ok
    assert _create_expr(E.EXPR_GRADIENT, coeffs=[0.5]) == E.S5D_EINVAL
    assert _create_expr(E.EXPR_GRADIENT, radius=2, coeffs=[0.5, 1.5]) == E.S5D_EINVAL
    assert _create_expr(E.EXPR_GRADIENT, box=True, coeffs=[0.5, 1.5]) == E.S5D_EINVAL
    assert _create_expr(E.EXPR_GRADIENT, ndim=3, interior=(8, 8, 8), coeffs=[0.5, 1.5]) == E.S5D_EINVAL
    assert _create_expr(E.EXPR_VARCOEF, coeffs=None) == ok
    assert _create_expr(E.EXPR_VARCOEF, coeffs=[0.2] * 5) == E.S5D_EINVAL
    assert _create_expr(E.EXPR_VARCOEF, ndim=3, interior=(8, 8, 8)) == E.S5D_EUNSUPPORTED
    assert _create_expr(E.EXPR_DIV, radius=4, coeffs=np.ones(18)) == E.S5D_EUNSUPPORTED
    assert _create_expr(E.EXPR_DIV, dtype=E.F32, accum=E.ACC_COMPENSATED,
                        coeffs=[1, 2, 3, 4, 5, 15]) == E.S5D_EUNSUPPORTED
    assert _create_expr(E.EXPR_DIV, coeffs=[1, 2, 3, 4, 5, 15],
                        tuning=_lib.make_tuning(kernel=2)) == E.S5D_EUNSUPPORTED
    assert _create_expr(7, coeffs=[1.0] * 5) == E.S5D_EINVAL


def test_run_fields_validation():
    lib = _lib.load()
    d, keep = _lib.make_desc(2, 1, False, _lib.F64, 0, (64, 64), 4, None, _lib.EXPR_VARCOEF)
    h = ctypes.c_void_p()
    assert lib.s5d_plan_create(ctypes.byref(d), None, ctypes.byref(h)) == _lib.S5D_OK
    idx = ctypes.c_int32()
    vp = ctypes.c_void_p
    # s5d_run refuses a plan with per-cell weights; s5d_run_fields needs them
    assert lib.s5d_run(h, vp(1 << 20), vp(1 << 28), None, ctypes.byref(idx)) == _lib.S5D_EINVAL
    assert lib.s5d_run_fields(h, vp(1 << 20), vp(1 << 28), None, None, ctypes.byref(idx)) == _lib.S5D_EINVAL
    assert lib.s5d_run_fields(h, vp(1 << 20), vp(1 << 28), vp((1 << 30) + 4), None,
                              ctypes.byref(idx)) == _lib.S5D_EINVAL  # misaligned
    lib.s5d_plan_destroy(h)
    st, h = _create(steps=0)
    assert st == _lib.S5D_OK
    # fields given for a plan without per-cell weights
    assert lib.s5d_run_fields(h, vp(1 << 20), vp(1 << 28), vp(1 << 30), None,
                              ctypes.byref(idx)) == _lib.S5D_EINVAL
    assert lib.s5d_run_fields(h, vp(1 << 20), vp(1 << 28), None, None, ctypes.byref(idx)) == _lib.S5D_OK
    lib.s5d_plan_destroy(h)


def test_waves_per_eu_is_reserved():
    st, _ = _create(tuning=_lib.make_tuning(waves_per_eu=2))
    assert st == _lib.S5D_EINVAL


@pytest.mark.parametrize("ndim,radius,box,dtype,accum,want", [
    (2, 1, False, _lib.F32, 1, "blocked"),   # compensated 5-point star: b_T = 3
    (2, 2, False, _lib.F32, 1, "direct"),    # other compensated 2D stencils: one step
    (2, 1, True, _lib.F32, 1, "direct"),
    (2, 4, True, _lib.F32, 0, "blocked"),    # float32 81-point box: blocked b_T = 1
    (2, 4, True, _lib.F64, 0, "blocked"),    # float64 81-point box: blocked b_T = 1
    (2, 1, False, _lib.F32, 0, "blocked"),
    (3, 1, True, _lib.F32, 1, "direct"),     # compensated 27-point box
    (3, 1, False, _lib.F32, 0, "blocked"),
])
def test_default_kernel_choice(ndim, radius, box, dtype, accum, want):
    """Which kernel family a plan without tuning takes.  A direct plan uploads
    its coefficients at creation, so without a GPU it ends in S5D_EDEVICE
    where a blocked plan succeeds; with a GPU the chosen family is queried."""
    lib = _lib.load()
    interior = (64, 64) if ndim == 2 else (16, 16, 16)
    st, h = _create(ndim=ndim, radius=radius, box=box, dtype=dtype, accum=accum, interior=interior)
    if st == _lib.S5D_OK:
        t = _lib.make_tuning()
        assert lib.s5d_plan_query(h, ctypes.byref(t), None) == _lib.S5D_OK
        lib.s5d_plan_destroy(h)
        assert t.kernel == _lib.KERNELS[want]
    else:
        assert want == "direct" and st == _lib.S5D_EDEVICE, _lib.last_error()
