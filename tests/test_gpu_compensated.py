"""GPU parity of the compensated float32 kernels (Dot2 accumulation).

The kernels and the oracle run the same error-free transformations in the same
canonical term order with contraction disabled, so the bar is bit-exact on
arbitrary inputs, not only on dyadic ones.  Coefficients carry random signs so
that the sums are ill-conditioned and compensated and plain accumulation give
different bits in many cells (checked, so that a plain kernel cannot pass).
"""
import numpy as np
import pytest

import oracle
import stencil_inputs as si
from geometry import compute_width
from gpu_util import run_gpu, say
from paper_2001_01473_amd import build as s5d_build

pytestmark = pytest.mark.gpu

V2 = [v for v in s5d_build.linear_variants_2d() if v[0] == 2]
V3 = [v for v in s5d_build.linear_variants_3d() if v[0] == 2]


def _signed_case(seed, ndim, r, box, interior, steps):
    case = si.make_case(seed, ndim, r, box, interior, steps)
    c32, g32 = case.as_dtype(np.float32)
    rng = np.random.default_rng(seed + 7)
    c32 = (c32 * np.where(rng.random(c32.size) < 0.5, -1, 1)).astype(np.float32)
    return c32, g32


def _check(g32, c32, r, box, T, **tuning):
    want = oracle.sweep(g32, radius=r, box=box, coeffs=c32, steps=T, accum="compensated")
    plain = oracle.sweep(g32, radius=r, box=box, coeffs=c32, steps=T)
    got, info = run_gpu(g32, radius=r, box=box, coeffs=c32.astype(np.float64), steps=T,
                        accum="compensated", **tuning)
    np.testing.assert_array_equal(got, want)
    if T > 0 and g32.size > 64:
        assert np.count_nonzero(got != plain) > 0
    return info


def _vid2(v):
    dtype, box, r, cpl, bt, nr = v
    return "f32c-%s%d-c%d-b%d" % ("box" if box else "star", r, cpl, bt)


def _vid3(v):
    dtype, box, r, cpl, m, nw, bt, nr = v
    return "f32c-%s%d-c%dm%dw%d-b%d" % ("box" if box else "star", r, cpl, m, nw, bt)


@pytest.mark.parametrize("v", V2, ids=[_vid2(v) for v in V2])
def test_comp2d_variant_bitwise(v):
    dtype, box, r, cpl, bt, nr = v
    C = compute_width(64 * cpl, bt, r, 4)
    interior = (3 * (19 + bt) + 5, 2 * C + C // 2 + 7)
    T = 2 * bt + 1
    c32, g32 = _signed_case(700 + bt, 2, r, bool(box), interior, T)
    say("comp2d", _vid2(v), interior, "T", T)
    info = _check(g32, c32, r, bool(box), T, bt=bt, cells_per_lane=cpl, stream_chunk=19 + bt)
    assert info["bt"] == bt


@pytest.mark.parametrize("v", V3, ids=[_vid3(v) for v in V3])
def test_comp3d_variant_bitwise(v):
    dtype, box, r, cpl, m, nw, bt, nr = v
    C1, C2 = nw * m - 2 * bt * r, compute_width(64 * cpl, bt, r, 4)
    chunk = 7 + bt
    interior = (2 * chunk + 3, 2 * C1 + C1 // 2 + 3, C2 + C2 // 3 + 5)
    T = 2 * bt + 1
    c32, g32 = _signed_case(800 + bt, 3, r, bool(box), interior, T)
    say("comp3d", _vid3(v), interior, "T", T)
    info = _check(g32, c32, r, bool(box), T, bt=bt, cells_per_lane=cpl, rows_per_wave=m,
                  stream_chunk=chunk)
    assert info["bt"] == bt


@pytest.mark.parametrize("ndim,r,box", [(2, 1, False), (2, 2, False), (2, 4, False),
                                        (2, 1, True), (2, 2, True), (3, 1, False),
                                        (3, 1, True), (3, 2, False)])
@pytest.mark.parametrize("T", [0, 1, 4, 7])
def test_comp_default_tuning(ndim, r, box, T):
    interior = (301, 517) if ndim == 2 else (37, 45, 150)
    c32, g32 = _signed_case(900 + T, ndim, r, box, interior, T)
    say("comp-default", ndim, r, box, T)
    _check(g32, c32, r, box, T)


@pytest.mark.parametrize("interior", [(1, 1), (3, 200), (70, 2), (1, 1, 1), (2, 7, 1), (9, 40, 3)])
def test_comp_tiny_grids(interior):
    ndim = len(interior)
    c32, g32 = _signed_case(41, ndim, 1, False, interior, 5)
    say("comp-tiny", interior)
    _check(g32, c32, 1, False, 5)


def test_comp_2048_full_compare():
    """2048^2 interior, 9-point star (radius 2), ten steps, default tuning:
    every cell bit-exact against the compensated oracle."""
    c32, g32 = _signed_case(si.workload_seed(9), 2, 2, False, (2048, 2048), 10)
    say("comp 2048^2 star r2 T=10")
    _check(g32, c32, 2, False, 10)

