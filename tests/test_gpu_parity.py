"""GPU parity: every compiled 2D kernel variant against the CPU oracle.

Bars (written in each test):
* dyadic inputs: bit-exact (every product and partial sum is exact, so the
  FMA-based kernel must equal the no-FMA oracle bit for bit);
* float64 random inputs: normwise and elementwise relative error <= 1e-12;
* float32 random inputs: error against the float64 oracle run on the same
  float32-rounded inputs within the a-priori bound T * (gamma_n + u) * max|A0|,
  with u = 2**-24 and gamma_n = n*u / (1 - n*u);
* temporal blocking: every b_T, stream-block length and cells-per-lane choice
  gives the same bits as b_T = 1.
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
VARIANTS = [v for v in s5d_build.linear_variants_2d() if v[0] != 2]
F64_TOL = 1e-12


def _vid(v):
    dtype, box, r, cpl, bt, nr = v
    return "%s-%s%d-c%d-b%d" % ("f32" if dtype == 0 else "f64", "box" if box else "star", r, cpl, bt)


def _geometry(v):
    """Interior extents spanning >= 2 tiles plus a ragged tail, and >= 3 stream
    blocks plus a ragged tail; the stream block may be shorter than the
    warm-up (b_T * r rows)."""
    dtype, box, r, cpl, bt, nr = v
    C = compute_width(64 * cpl, bt, r, 4 if dtype == 0 else 8)
    I1 = 2 * C + C // 2 + 7
    chunk = 19 + bt
    I0 = 3 * chunk + 5
    return (I0, I1), chunk


def _np_dtype(v):
    return np.float32 if v[0] == 0 else np.float64


@pytest.mark.parametrize("v", VARIANTS, ids=[_vid(v) for v in VARIANTS])
def test_variant_dyadic_bitwise(v):
    dtype, box, r, cpl, bt, nr = v
    dt = _np_dtype(v)
    (I0, I1), chunk = _geometry(v)
    bits = 24 if dt == np.float32 else 53
    case = si.make_dyadic_case(100 + bt, 2, r, bool(box), (I0, I1), 1)
    tmax = si.max_exact_steps(case.meta["q"], case.meta["m"], bits)
    T = min(tmax, 2 * bt + 1)
    want = oracle.sweep(case.grid.astype(dt), radius=r, box=bool(box),
                        coeffs=case.coeffs.astype(dt), steps=T)
    say("dyadic", _vid(v), "interior", (I0, I1), "T", T, "chunk", chunk)
    got, info = run_gpu(case.grid.astype(dt), radius=r, box=bool(box),
                        coeffs=case.coeffs, steps=T, bt=bt, cells_per_lane=cpl,
                        stream_chunk=chunk)
    assert info["bt"] == min(bt, T)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("v", VARIANTS, ids=[_vid(v) for v in VARIANTS])
def test_variant_random_parity(v):
    dtype, box, r, cpl, bt, nr = v
    dt = _np_dtype(v)
    (I0, I1), chunk = _geometry(v)
    T = 2 * bt + 3
    case = si.make_case(200 + bt, 2, r, bool(box), (I0, I1), T)
    c_in, g_in = case.as_dtype(dt)
    ref = oracle.sweep(g_in.astype(np.float64), radius=r, box=bool(box),
                       coeffs=c_in.astype(np.float64), steps=T)
    say("random", _vid(v), "interior", (I0, I1), "T", T)
    got, _ = run_gpu(g_in, radius=r, box=bool(box), coeffs=case.coeffs, steps=T,
                     bt=bt, cells_per_lane=cpl, stream_chunk=chunk)
    base, _ = run_gpu(g_in, radius=r, box=bool(box), coeffs=case.coeffs, steps=T,
                      bt=1, cells_per_lane=cpl, stream_chunk=chunk)
    np.testing.assert_array_equal(got, base)
    norm, elem = rel_errors(got, ref)
    if dt == np.float64:
        assert norm <= F64_TOL and elem <= F64_TOL, (norm, elem)
    else:
        n = len(c_in)
        bound = T * (pins.gamma(n, pins.U32) + pins.U32) * float(np.max(g_in)) * 1.01
        assert float(np.max(np.abs(got.astype(np.float64) - ref))) <= bound


@pytest.mark.parametrize("dt", [np.float32, np.float64])
@pytest.mark.parametrize("r,box", [(1, False), (2, False), (4, False), (1, True), (2, True)])
@pytest.mark.parametrize("interior", [(1, 1), (1, 6), (6, 1), (2, 3), (7, 9), (3, 300)])
def test_tiny_and_degenerate_grids(dt, r, box, interior):
    T = 7
    case = si.make_dyadic_case(7, 2, r, box, interior, T, m=1)
    bits = 24 if dt == np.float32 else 53
    T = min(T, si.max_exact_steps(case.meta["q"], case.meta["m"], bits))
    want = oracle.sweep(case.grid.astype(dt), radius=r, box=box, coeffs=case.coeffs.astype(dt),
                        steps=T)
    say("tiny", dt.__name__, r, box, interior, T)
    got, _ = run_gpu(case.grid.astype(dt), radius=r, box=box, coeffs=case.coeffs, steps=T)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("T", [0, 1, 2, 3, 4, 5, 7, 8, 9, 13])
def test_round_parity_and_remainders(T):
    """Result lands in buffer T % 2 for every remainder of T mod b_T."""
    case = si.make_case(31, 2, 1, False, (70, 300), T)
    ref = oracle.sweep(case.grid, radius=1, box=False, coeffs=case.coeffs, steps=T)
    say("parity T", T)
    got, info = run_gpu(case.grid, radius=1, box=False, coeffs=case.coeffs, steps=T,
                        bt=4, stream_chunk=16)
    norm, elem = rel_errors(got, ref)
    assert norm <= F64_TOL and elem <= F64_TOL


def test_blocking_invariance_f64():
    """b_T, h_SN and cells-per-lane choices give identical bits."""
    case = si.make_case(41, 2, 2, False, (211, 777), 24)
    built = {(v[3], v[4]) for v in VARIANTS if v[:3] == (1, 0, 2)}
    wanted = [(1, 4, 64), (2, 2, 17), (3, 4, 500), (4, 4, 9), (6, 2, 33),
              (8, 2, 250), (10, 2, 40), (4, 2, 211), (5, 4, 31), (7, 2, 12)]
    configs = [(bt, cpl, ch) for bt, cpl, ch in wanted if (cpl, bt) in built]
    assert len(configs) >= 6, configs
    outs = []
    for bt, cpl, chunk in configs:
        say("invariance", bt, cpl, chunk)
        got, info = run_gpu(case.grid, radius=2, box=False, coeffs=case.coeffs, steps=24,
                            bt=bt, cells_per_lane=cpl, stream_chunk=chunk)
        outs.append(got)
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])
    ref = oracle.sweep(case.grid, radius=2, box=False, coeffs=case.coeffs, steps=24)
    norm, elem = rel_errors(outs[0], ref)
    assert norm <= F64_TOL and elem <= F64_TOL


def test_default_tuning_matches_oracle():
    for (r, box, dt) in [(1, False, np.float32), (3, False, np.float64), (2, True, np.float32)]:
        case = si.make_case(51, 2, r, box, (333, 1031), 25)
        c_in, g_in = case.as_dtype(dt)
        ref = oracle.sweep(g_in.astype(np.float64), radius=r, box=box,
                           coeffs=c_in.astype(np.float64), steps=25)
        say("default tuning", r, box, dt.__name__)
        got, info = run_gpu(g_in, radius=r, box=box, coeffs=case.coeffs, steps=25)
        norm, elem = rel_errors(got, ref)
        tol = F64_TOL if dt == np.float64 else 25 * (len(c_in) + 2) * pins.U32
        assert norm <= tol, (info, norm)


def test_cfg0_full_512_f64_plain():
    """512^2 interior, 5-point star, float64, 100 steps, b_T = 1 (plain sweep)."""
    case = si.make_case(si.workload_seed(0), 2, 1, False, (512, 512), 100)
    ref = oracle.sweep(case.grid, radius=1, box=False, coeffs=case.coeffs, steps=100)
    say("cfg0 512^2 f64 T=100 bt=1")
    got, info = run_gpu(case.grid, radius=1, box=False, coeffs=case.coeffs, steps=100, bt=1)
    norm, elem = rel_errors(got, ref)
    assert norm <= F64_TOL and elem <= F64_TOL, (norm, elem)


def _crop_check(got, grid, coeffs, r, box, T, points):
    """Sampled outputs: the oracle on a window of half-width (T+1)*r+1 around each
    point; cells outside the window cannot reach the point within T steps."""
    H = (T + 1) * r + 1
    for p in points:
        lo = [max(0, p[a] - H) for a in range(2)]
        hi = [min(grid.shape[a], p[a] + H + 1) for a in range(2)]
        win = grid[lo[0]:hi[0], lo[1]:hi[1]].astype(np.float64)
        out = oracle.sweep(win, radius=r, box=box, coeffs=coeffs, steps=T)
        want = out[p[0] - lo[0], p[1] - lo[1]]
        g = float(got[p])
        assert abs(g - want) <= F64_TOL * max(abs(want), 1e-300) or (
            got.dtype == np.float32 and abs(g - want) <= T * (len(coeffs) + 2) * pins.U32), (p, g, want)


@pytest.mark.parametrize("dt,r,box", [(np.float32, 1, False), (np.float64, 1, False),
                                      (np.float32, 2, True)])
def test_full_size_16384_sampled(dt, r, box):
    """16384^2 interior in the launch configuration the benchmark uses (library
    default tuning), a short sweep of several rounds: sampled cells against the
    windowed oracle, b_T-invariance against b_T = 1 and the maximum principle."""
    import torch
    N = 16384
    case = si.make_case(si.workload_seed(1), 2, r, box, (N, N), 1)
    c_in, g_in = case.as_dtype(dt)
    say("full-size", dt.__name__, r, box)
    got, info = run_gpu(g_in, radius=r, box=box, coeffs=case.coeffs, steps=1)
    T = 2 * info["bt"] + 1
    got, info = run_gpu(g_in, radius=r, box=box, coeffs=case.coeffs, steps=T)
    P = N + 2 * r
    rng = np.random.default_rng(5)
    pts = [(r, r), (r, P - r - 1), (P - r - 1, r), (P - r - 1, P - r - 1), (P // 2, P // 2)]
    pts += [(int(a), int(b)) for a, b in rng.integers(r, P - r, size=(11, 2))]
    _crop_check(got, g_in, c_in.astype(np.float64), r, box, T, pts)
    assert got.min() >= g_in.min() - 1e-6 and got.max() <= g_in.max() + 1e-6
    base, _ = run_gpu(g_in, radius=r, box=box, coeffs=case.coeffs, steps=T, bt=1)
    np.testing.assert_array_equal(got, base)
    del base, got
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_full_size_16384_streaming_bt1(dt):
    """16384^2 interior at b_T = 1, the launch the benchmark's b_T = 1 point
    times (the row-streaming kernel): the same bits as the blocked kernel at
    b_T = 1, sampled cells against the windowed oracle."""
    N, r, T = 16384, 1, 3
    case = si.make_case(si.workload_seed(1), 2, r, False, (N, N), T)
    c_in, g_in = case.as_dtype(dt)
    say("full-size streaming b_T=1", dt.__name__)
    got, info = run_gpu(g_in, radius=r, box=False, coeffs=case.coeffs, steps=T, bt=1)
    assert info["kernel"] == 2
    base, binfo = run_gpu(g_in, radius=r, box=False, coeffs=case.coeffs, steps=T, bt=1, kernel="blocked")
    assert binfo["kernel"] == 1
    np.testing.assert_array_equal(got, base)
    P = N + 2 * r
    rng = np.random.default_rng(9)
    pts = [(r, r), (r, P - r - 1), (P - r - 1, r), (P - r - 1, P - r - 1), (P // 2, P // 2)]
    pts += [(int(a), int(b)) for a, b in rng.integers(r, P - r, size=(11, 2))]
    _crop_check(got, g_in, c_in.astype(np.float64), r, False, T, pts)
