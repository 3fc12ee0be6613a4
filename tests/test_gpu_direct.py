"""GPU parity of the direct (one step per launch) kernels.

They cover every radius 1..4 and shape in 2D and 3D, in all three kernel
kinds.  Bars: dyadic inputs bit-exact against the oracle; float64 random
inputs within 1e-12 (normwise and elementwise); compensated float32
bit-exact against the compensated oracle on arbitrary inputs; and, where a
temporally blocked variant exists too, the same bits as that variant (the
terms are summed in the same canonical order with the same operations).
Grids span several tiles on every axis with ragged tails.
"""
import numpy as np
import pytest

import oracle
import stencil_inputs as si
from gpu_util import rel_errors, run_gpu, say

pytestmark = pytest.mark.gpu

STENCILS = [(nd, r, box) for nd in (2, 3) for r in (1, 2, 3, 4) for box in (False, True)]


def _interior(nd, r):
    if nd == 2:
        return (2 * 16 + 5, 2 * 64 + 11)
    return (2 * 4 + 3, 2 * 8 + 3, (32 if r >= 3 else 64) + 9)


def _sid(s):
    nd, r, box = s
    return "%s%dd%dr" % ("box" if box else "star", nd, r)


@pytest.mark.parametrize("s", STENCILS, ids=[_sid(s) for s in STENCILS])
@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_direct_dyadic_bitwise(s, dt):
    nd, r, box = s
    case = si.make_dyadic_case(31 + r, nd, r, box, _interior(nd, r), 1, m=2)
    bits = 24 if dt == np.float32 else 53
    T = max(1, min(3, si.max_exact_steps(case.meta["q"], case.meta["m"], bits)))
    want = oracle.sweep(case.grid.astype(dt), radius=r, box=box, coeffs=case.coeffs.astype(dt), steps=T)
    say("direct dyadic", _sid(s), dt.__name__, "T", T)
    got, info = run_gpu(case.grid.astype(dt), radius=r, box=box, coeffs=case.coeffs, steps=T,
                        kernel="direct")
    assert info["kernel"] == 2 and info["bt"] == 1
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("s", STENCILS, ids=[_sid(s) for s in STENCILS])
def test_direct_f64_random(s):
    nd, r, box = s
    T = 4
    case = si.make_case(41 + r, nd, r, box, _interior(nd, r), T)
    ref = oracle.sweep(case.grid, radius=r, box=box, coeffs=case.coeffs, steps=T)
    say("direct f64", _sid(s))
    got, _ = run_gpu(case.grid, radius=r, box=box, coeffs=case.coeffs, steps=T, kernel="direct")
    norm, elem = rel_errors(got, ref)
    assert norm <= 1e-12 and elem <= 1e-12, (norm, elem)


@pytest.mark.parametrize("s", STENCILS, ids=[_sid(s) for s in STENCILS])
def test_direct_compensated_bitwise(s):
    nd, r, box = s
    T = 3
    case = si.make_case(51 + r, nd, r, box, _interior(nd, r), T)
    c32, g32 = case.as_dtype(np.float32)
    rng = np.random.default_rng(52 + r)
    c32 = (c32 * np.where(rng.random(c32.size) < 0.5, -1, 1)).astype(np.float32)
    want = oracle.sweep(g32, radius=r, box=box, coeffs=c32, steps=T, accum="compensated")
    say("direct f32c", _sid(s))
    got, _ = run_gpu(g32, radius=r, box=box, coeffs=c32.astype(np.float64), steps=T,
                     accum="compensated", kernel="direct")
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("kind", ["f32", "f64", "f32c"])
@pytest.mark.parametrize("s", [(2, 1, False), (2, 2, True), (2, 4, False), (3, 1, False),
                               (3, 1, True), (3, 2, False)], ids=_sid)
def test_direct_equals_blocked(kind, s):
    nd, r, box = s
    dt = np.float64 if kind == "f64" else np.float32
    accum = "compensated" if kind == "f32c" else "plain"
    T = 5
    interior = (70, 300) if nd == 2 else (19, 37, 150)
    case = si.make_case(61 + r, nd, r, box, interior, T)
    c_in, g_in = case.as_dtype(dt)
    say("direct vs blocked", kind, _sid(s))
    a, ia = run_gpu(g_in, radius=r, box=box, coeffs=case.coeffs, steps=T, accum=accum,
                    kernel="direct")
    b, ib = run_gpu(g_in, radius=r, box=box, coeffs=case.coeffs, steps=T, accum=accum,
                    kernel="blocked")
    assert ia["kernel"] == 2 and ib["kernel"] == 1
    np.testing.assert_array_equal(a, b)


def test_auto_falls_back_to_direct():
    """The float64 125-point box (3D, radius 2) has no blocked variant: the
    default plan takes the direct kernels and is within 1e-12 of the oracle."""
    case = si.make_case(71, 3, 2, True, (21, 30, 100), 3)
    ref = oracle.sweep(case.grid, radius=2, box=True, coeffs=case.coeffs, steps=3)
    got, info = run_gpu(case.grid, radius=2, box=True, coeffs=case.coeffs, steps=3)
    assert info["kernel"] == 2
    assert max(rel_errors(got, ref)) <= 1e-12


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("s", [(2, 1, False), (2, 2, False), (2, 3, False), (2, 4, False), (2, 1, True),
                               (2, 2, True)], ids=_sid)
def test_row_streaming_spans_segments(s, dt):
    """The row-streaming kernel on rows of several workgroup segments (512
    threads x one 16-byte vector) plus a ragged tail, on a row shorter than
    one wave, and on row counts that leave a thread's group of 2 or 4 rows
    partly empty (1, 3, 6, 13 rows): the same bits as the blocked kernel at
    b_T = 1, and float64 within 1e-12 of the oracle."""
    nd, r, box = s
    seg = 512 * (16 // np.dtype(dt).itemsize)
    T = 3
    for interior in ((13, 2 * seg + 389), (6, 37), (1, 70), (3, seg + 3)):
        case = si.make_case(91 + r, nd, r, box, interior, T)
        c_in, g_in = case.as_dtype(dt)
        say("row streaming", _sid(s), dt.__name__, interior)
        a, ia = run_gpu(g_in, radius=r, box=box, coeffs=case.coeffs, steps=T, bt=1)
        b, ib = run_gpu(g_in, radius=r, box=box, coeffs=case.coeffs, steps=T, bt=1, kernel="blocked")
        assert ia["kernel"] == 2 and ib["kernel"] == 1
        np.testing.assert_array_equal(a, b)
        if dt == np.float64:
            ref = oracle.sweep(g_in, radius=r, box=box, coeffs=c_in, steps=T)
            assert max(rel_errors(a, ref)) <= 1e-12


@pytest.mark.parametrize("kind", ["f32", "f64", "f32c"])
@pytest.mark.parametrize("r,box", [(1, False), (2, False), (3, False), (4, False), (1, True)],
                         ids=["star1", "star2", "star3", "star4", "box1"])
def test_row_streaming_3d_spans_segments(kind, r, box):
    """The 3D row-streaming kernel (stars, 27-point box) on rows of several wave
    segments (64 lanes x one 16-byte vector) plus a ragged tail, on rows
    shorter than one wave, and on row counts that leave a wave's group of
    2 or 4 rows partly empty (1, 3, 6, 7 rows): the same bits as the blocked
    kernel at b_T = 1 (radius 1-2, where one is built), float64 within 1e-12
    of the oracle, compensated float32 bit-exact against the compensated
    oracle."""
    dt = np.float64 if kind == "f64" else np.float32
    accum = "compensated" if kind == "f32c" else "plain"
    seg = 64 * (16 // np.dtype(dt).itemsize)
    T = 2
    for interior in ((5, 7, 2 * seg + 77), (4, 3, 19), (3, 1, seg + 5), (2, 6, 40)):
        case = si.make_case(97 + r, 3, r, box, interior, T)
        c_in, g_in = case.as_dtype(dt)
        say("3D row streaming", kind, "r", r, "box", box, interior)
        a, ia = run_gpu(g_in, radius=r, box=box, coeffs=case.coeffs, steps=T, accum=accum, kernel="direct")
        assert ia["kernel"] == 2
        if r <= 2:
            b, ib = run_gpu(g_in, radius=r, box=box, coeffs=case.coeffs, steps=T, accum=accum,
                            kernel="blocked", bt=1)
            np.testing.assert_array_equal(a, b)
        if kind == "f64":
            ref = oracle.sweep(g_in, radius=r, box=box, coeffs=c_in, steps=T)
            assert max(rel_errors(a, ref)) <= 1e-12
        elif kind == "f32c":
            want = oracle.sweep(g_in, radius=r, box=box, coeffs=c_in, steps=T, accum="compensated")
            np.testing.assert_array_equal(a, want)
