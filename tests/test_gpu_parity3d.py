"""GPU parity of the 3D kernels against the CPU oracle.

Bars, as for 2D: bit-exact on dyadic inputs; float64 random inputs within
1e-12 relative (normwise and elementwise); float32 random inputs within
T * (gamma_n + u) * max|A0| of the float64 oracle on the same rounded inputs;
every b_T bit-identical to b_T = 1.  Grids span several tiles with ragged
tails on both in-plane axes and several stream blocks along axis 0.
"""
import numpy as np
import pytest

import oracle
import pins
import stencil_inputs as si
from geometry import compute_width
from gpu_util import rel_errors, run_gpu, say
from paper_2001_01473_amd import build as s5d_build

pytestmark = pytest.mark.gpu

# plain accumulation only; the compensated kernels have their own tests
VARIANTS = [v for v in s5d_build.linear_variants_3d() if v[0] != 2]
F64_TOL = 1e-12


def _vid(v):
    dtype, box, r, cpl, m, nw, bt, nr = v
    return "%s-%s%d-c%dm%dw%d-b%d" % ("f32" if dtype == 0 else "f64", "box" if box else "star",
                                       r, cpl, m, nw, bt)


def _geometry(v):
    dtype, box, r, cpl, m, nw, bt, nr = v
    C1 = nw * m - 2 * bt * r
    C2 = compute_width(64 * cpl, bt, r, 4 if dtype != 1 else 8)
    I1 = 2 * C1 + C1 // 2 + 3
    I2 = C2 + C2 // 3 + 5
    chunk = 7 + bt
    I0 = 2 * chunk + 3
    return (I0, I1, I2), chunk


def _dt(v):
    return np.float32 if v[0] == 0 else np.float64


@pytest.mark.parametrize("v", VARIANTS, ids=[_vid(v) for v in VARIANTS])
def test_variant3d_dyadic_bitwise(v):
    dtype, box, r, cpl, m, nw, bt, nr = v
    dt = _dt(v)
    interior, chunk = _geometry(v)
    bits = 24 if dt == np.float32 else 53
    case = si.make_dyadic_case(300 + bt, 3, r, bool(box), interior, 1)
    T = min(si.max_exact_steps(case.meta["q"], case.meta["m"], bits), 2 * bt + 1)
    want = oracle.sweep(case.grid.astype(dt), radius=r, box=bool(box),
                        coeffs=case.coeffs.astype(dt), steps=T)
    say("dyadic3d", _vid(v), interior, "T", T, "chunk", chunk)
    got, info = run_gpu(case.grid.astype(dt), radius=r, box=bool(box), coeffs=case.coeffs,
                        steps=T, bt=bt, cells_per_lane=cpl, rows_per_wave=m, stream_chunk=chunk)
    assert info["bt"] == min(bt, T)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("v", VARIANTS, ids=[_vid(v) for v in VARIANTS])
def test_variant3d_random_parity(v):
    dtype, box, r, cpl, m, nw, bt, nr = v
    dt = _dt(v)
    interior, chunk = _geometry(v)
    T = 2 * bt + 1
    case = si.make_case(400 + bt, 3, r, bool(box), interior, T)
    c_in, g_in = case.as_dtype(dt)
    ref = oracle.sweep(g_in.astype(np.float64), radius=r, box=bool(box),
                       coeffs=c_in.astype(np.float64), steps=T)
    say("random3d", _vid(v), interior, "T", T)
    kw = dict(cells_per_lane=cpl, rows_per_wave=m, stream_chunk=chunk)
    got, _ = run_gpu(g_in, radius=r, box=bool(box), coeffs=case.coeffs, steps=T, bt=bt, **kw)
    base, _ = run_gpu(g_in, radius=r, box=bool(box), coeffs=case.coeffs, steps=T, bt=1, **kw)
    np.testing.assert_array_equal(got, base)
    norm, elem = rel_errors(got, ref)
    if dt == np.float64:
        assert norm <= F64_TOL and elem <= F64_TOL, (norm, elem)
    else:
        n = len(c_in)
        bound = T * (pins.gamma(n, pins.U32) + pins.U32) * float(np.max(g_in)) * 1.01
        assert float(np.max(np.abs(got.astype(np.float64) - ref))) <= bound


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("r,box", [(1, False), (1, True), (2, False), (2, True)])
@pytest.mark.parametrize("interior", [(1, 1, 1), (3, 1, 5), (2, 7, 1), (4, 5, 6), (9, 40, 3)])
def test_tiny_and_degenerate_grids_3d(dt, r, box, interior):
    # (a stencil without a blocked variant runs on the direct kernels)
    case = si.make_dyadic_case(17, 3, r, box, interior, 5, m=1)
    bits = 24 if dt == np.float32 else 53
    T = min(5, si.max_exact_steps(case.meta["q"], case.meta["m"], bits))
    want = oracle.sweep(case.grid.astype(dt), radius=r, box=box, coeffs=case.coeffs.astype(dt),
                        steps=T)
    say("tiny3d", dt.__name__, r, box, interior, T)
    got, _ = run_gpu(case.grid.astype(dt), radius=r, box=box, coeffs=case.coeffs, steps=T)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("dt,box", [(np.float64, False), (np.float64, True), (np.float32, False)])
def test_3d_default_tuning_and_remainders(dt, box):
    for T in (1, 2, 5, 8):
        case = si.make_case(500 + T, 3, 1, box, (37, 45, 150), T)
        c_in, g_in = case.as_dtype(dt)
        ref = oracle.sweep(g_in.astype(np.float64), radius=1, box=box,
                           coeffs=c_in.astype(np.float64), steps=T)
        say("default3d", dt.__name__, box, T)
        got, info = run_gpu(g_in, radius=1, box=box, coeffs=case.coeffs, steps=T)
        norm, elem = rel_errors(got, ref)
        tol = F64_TOL if dt == np.float64 else T * (len(c_in) + 2) * pins.U32
        assert norm <= tol, (info, norm)


def test_3d_full_size_512_sampled():
    """512^3 interior, 7-point star, float64, default tuning, a short sweep of
    several rounds: sampled cells against the windowed oracle, b_T-invariance
    against b_T = 1 and the maximum principle."""
    N = 512
    case = si.make_case(si.workload_seed(2), 3, 1, False, (N, N, N), 1)
    say("full-size 3d 512^3 f64")
    got, info = run_gpu(case.grid, radius=1, box=False, coeffs=case.coeffs, steps=1)
    T = 2 * info["bt"] + 1
    got, info = run_gpu(case.grid, radius=1, box=False, coeffs=case.coeffs, steps=T)
    P = N + 2
    rng = np.random.default_rng(6)
    pts = [(1, 1, 1), (P - 2, P - 2, P - 2), (1, P // 2, P - 2), (P // 2, P // 2, P // 2)]
    pts += [tuple(int(x) for x in rng.integers(1, P - 1, size=3)) for _ in range(8)]
    H = (T + 1) + 1
    for p in pts:
        lo = [max(0, p[a] - H) for a in range(3)]
        hi = [min(P, p[a] + H + 1) for a in range(3)]
        win = case.grid[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]]
        want = oracle.sweep(win, radius=1, box=False, coeffs=case.coeffs, steps=T)[
            p[0] - lo[0], p[1] - lo[1], p[2] - lo[2]]
        assert abs(float(got[p]) - want) <= F64_TOL * abs(want), (p, float(got[p]), want)
    assert got.min() >= case.grid.min() - 1e-12 and got.max() <= case.grid.max() + 1e-12
    base, _ = run_gpu(case.grid, radius=1, box=False, coeffs=case.coeffs, steps=T, bt=1)
    np.testing.assert_array_equal(got, base)
