"""GPU parity of the expression and variable-coefficient stencils (AN5D
Table 3's general benchmarks: j2d5pt, j2d9pt, j2d9pt-gol, j3d27pt as a
weighted sum divided by c0, gradient2d; and per-cell weights) against the CPU
oracle.

Bars:
* weighted sum / c0 and per-cell weights on dyadic inputs (integer weights,
  power-of-two divisor, or per-cell weights k/2^q): bit-exact, every compiled
  variant, on grids of >= 2 tiles plus a ragged tail and >= 3 stream blocks;
* the same on random inputs: float64 normwise and elementwise relative error
  <= 1e-12; float32 against the float64 oracle on the same rounded inputs
  within T*(gamma_{n+1} + u)*max|A0|;
* gradient2d: bit-exact against the oracle in float64 and float32 on random
  inputs (both evaluate the same IEEE operations in the same order, with
  correctly rounded square root and division);
* every depth gives the bits of depth 1; a batch of division plans gives the
  bits of single runs; window plans are refused by batches and s5d_run.
"""
import numpy as np
import pytest

import oracle
import paper_2001_01473_amd as s5d
import pins
import stencil_inputs as si
from geometry import compute_width
from gpu_util import rel_errors, say, torch
from paper_2001_01473_amd import build as s5d_build

pytestmark = pytest.mark.gpu

EXPR_NAMES = {1: "div", 2: "gradient", 3: "varcoef"}
V2 = [v for v in s5d_build.variants_2d() if v[1] != 0]
V3 = [v for v in s5d_build.variants_3d() if v[1] != 0]


def _vid(v):
    dtype, expr, box, r, cpl, bt, nr = v
    return "%s-%s-%s%d-c%d-b%d" % ("f32" if dtype == 0 else "f64", EXPR_NAMES[expr],
                                   "box" if box else "star", r, cpl, bt)


def _vid3(v):
    dtype, expr, box, r, cpl, m, nw, bt, nr = v
    return "%s-%s-%s%d-c%dm%dw%d-b%d" % ("f32" if dtype == 0 else "f64", EXPR_NAMES[expr],
                                         "box" if box else "star", r, cpl, m, nw, bt)


def _geometry(v):
    dtype, expr, box, r, cpl, bt, nr = v
    C = compute_width(64 * cpl, bt, r, 4 if dtype == 0 else 8)
    chunk = 19 + bt
    return (3 * chunk + 5, 2 * C + C // 2 + 7), chunk


def _run(grid, plan, fields=None):
    t = torch()
    x = t.from_numpy(np.ascontiguousarray(grid)).to("cuda:0")
    y = t.empty_like(x)
    f = None if fields is None else t.from_numpy(np.ascontiguousarray(fields)).to("cuda:0")
    idx = plan.run(x, y, fields=f)
    t.cuda.synchronize()
    out = (x if idx == 0 else y).cpu().numpy()
    assert idx == plan.steps % 2
    return out


def _plan(v_expr, dt, interior, r, box, T, coeffs, **tuning):
    return s5d.Plan(ndim=len(interior), radius=r, box=box, dtype=dt, interior=interior, steps=T,
                    coeffs=coeffs, expr=EXPR_NAMES[v_expr], **tuning)


def _dyadic_weights(rng, n, q):
    """n non-negative integers summing to 2^q (none of them all of it)."""
    while True:
        cuts = np.sort(rng.integers(0, 2 ** q + 1, size=n - 1))
        w = np.diff(np.concatenate([[0], cuts, [2 ** q]]))
        if w.max() < 2 ** q:
            return w


@pytest.mark.parametrize("v", V2, ids=[_vid(v) for v in V2])
def test_expr_variant_exact(v):
    """Dyadic (div, varcoef) or random (gradient) inputs: the oracle's bits."""
    dtype, expr, box, r, cpl, bt, nr = v
    dt = np.float32 if dtype == 0 else np.float64
    bits = 24 if dtype == 0 else 53
    interior, chunk = _geometry(v)
    n = si.n_points(2, r, bool(box))
    rng = np.random.default_rng(400 + 10 * expr + bt)
    say("expr exact", _vid(v), interior, "chunk", chunk)
    tune = dict(bt=bt, cells_per_lane=cpl, stream_chunk=chunk)
    if expr == 2:
        T = 2 * bt + 3
        grid = rng.random(si.padded_shape(interior, 1)).astype(dt)
        cc, c0 = dt(rng.random() / 2), dt(1 + rng.random())
        want = oracle.sweep_gradient(grid, cc=cc, c0=c0, steps=T)
        plan = _plan(2, dt, interior, 1, False, T, [float(cc), float(c0)], **tune)
        got = _run(grid, plan)
    else:
        q, m = 4, 4
        T = min(2 * bt + 1, (bits - m) // q)
        x = rng.integers(0, 2 ** m, size=si.padded_shape(interior, r))
        grid = np.ldexp(x.astype(np.float64), -m).astype(dt)
        if expr == 1:
            w = _dyadic_weights(rng, n, q).astype(np.float64)
            want = oracle.sweep_div(grid, radius=r, box=bool(box), coeffs=w.astype(dt), divisor=dt(2 ** q),
                                    steps=T)
            plan = _plan(1, dt, interior, r, bool(box), T, list(w) + [2.0 ** q], **tune)
            got = _run(grid, plan)
        else:
            cf = np.stack([_dyadic_weights(rng, n, q) for _ in range(int(np.prod(interior)))], axis=1)
            cf = np.ldexp(cf.reshape((n,) + interior).astype(np.float64), -q).astype(dt)
            want = oracle.sweep_varcoef(grid, radius=r, box=bool(box), cfield=cf, steps=T)
            plan = _plan(3, dt, interior, r, bool(box), T, None, **tune)
            got = _run(grid, plan, cf)
    assert plan.query()["bt"] == min(bt, T)
    plan.close()
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("v", [v for v in V2 if v[1] != 2], ids=[_vid(v) for v in V2 if v[1] != 2])
def test_expr_variant_random(v):
    dtype, expr, box, r, cpl, bt, nr = v
    dt = np.float32 if dtype == 0 else np.float64
    interior, chunk = _geometry(v)
    n = si.n_points(2, r, bool(box))
    T = 2 * bt + 3
    rng = np.random.default_rng(500 + 10 * expr + bt)
    grid = rng.random(si.padded_shape(interior, r))
    tune = dict(bt=bt, cells_per_lane=cpl, stream_chunk=chunk)
    say("expr random", _vid(v), interior)
    g_in = grid.astype(dt)
    if expr == 1:
        u = rng.random(n)
        c0 = float(u.sum())
        ref = oracle.sweep_div(g_in.astype(np.float64), radius=r, box=bool(box),
                               coeffs=u.astype(dt).astype(np.float64), divisor=float(dt(c0)), steps=T)
        plan = _plan(1, dt, interior, r, bool(box), T, list(u) + [c0], **tune)
        got = _run(g_in, plan)
    else:
        u = rng.random((n,) + interior)
        cf = (u / u.sum(axis=0)).astype(dt)
        ref = oracle.sweep_varcoef(g_in.astype(np.float64), radius=r, box=bool(box),
                                   cfield=cf.astype(np.float64), steps=T)
        plan = _plan(3, dt, interior, r, bool(box), T, None, **tune)
        got = _run(g_in, plan, cf)
    plan.close()
    if dt == np.float64:
        norm, elem = rel_errors(got, ref)
        assert norm <= 1e-12 and elem <= 1e-12, (norm, elem)
    else:
        bound = T * (pins.gamma(n + 1, pins.U32) + pins.U32) * float(g_in.max()) * 1.01
        assert float(np.max(np.abs(got.astype(np.float64) - ref))) <= bound


@pytest.mark.parametrize("v", V3, ids=[_vid3(v) for v in V3])
def test_j3d27pt_variant(v):
    """The 27-point box divided by c0: dyadic bit-exact, random float64 within
    1e-12."""
    dtype, expr, box, r, cpl, m, nw, bt, nr = v
    dt = np.float32 if dtype == 0 else np.float64
    bits = 24 if dtype == 0 else 53
    C1 = nw * m - 2 * bt * r
    C2 = compute_width(64 * cpl, bt, r, 4 if dtype == 0 else 8)
    chunk = 7 + bt
    interior = (2 * chunk + 3, 2 * C1 + C1 // 2 + 3, C2 + C2 // 3 + 5)
    rng = np.random.default_rng(600 + bt)
    q, mm = 5, 4
    T = min(2 * bt + 1, (bits - mm) // q)
    x = rng.integers(0, 2 ** mm, size=si.padded_shape(interior, 1))
    grid = np.ldexp(x.astype(np.float64), -mm).astype(dt)
    w = _dyadic_weights(rng, 27, q).astype(np.float64)
    tune = dict(bt=bt, cells_per_lane=cpl, rows_per_wave=m, stream_chunk=chunk)
    say("j3d27pt", _vid3(v), interior, "T", T)
    want = oracle.sweep_div(grid, radius=1, box=True, coeffs=w.astype(dt), divisor=dt(2 ** q), steps=T)
    plan = _plan(1, dt, interior, 1, True, T, list(w) + [2.0 ** q], **tune)
    np.testing.assert_array_equal(_run(grid, plan), want)
    plan.close()
    if dt == np.float64:
        T = 2 * bt + 1
        g = rng.random(si.padded_shape(interior, 1))
        u = rng.random(27)
        ref = oracle.sweep_div(g, radius=1, box=True, coeffs=u, divisor=float(u.sum()), steps=T)
        plan = _plan(1, dt, interior, 1, True, T, list(u) + [float(u.sum())], **tune)
        assert max(rel_errors(_run(g, plan), ref)) <= 1e-12
        plan.close()


@pytest.mark.parametrize("expr,r,box", [(1, 1, False), (1, 2, False), (1, 1, True), (2, 1, False),
                                        (3, 1, False), (3, 1, True)])
@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_expr_depths_same_bits_default_plan_and_degenerate(expr, r, box, dt):
    """Every compiled depth gives depth 1's bits on random inputs; the default
    plan too; tiny grids and T = 0 work."""
    interior = (101, 333)
    n = si.n_points(2, r, box)
    rng = np.random.default_rng(700 + expr)
    grid = rng.random(si.padded_shape(interior, r)).astype(dt)
    coeffs = None
    fields = None
    if expr == 1:
        u = rng.random(n)
        coeffs = list(u) + [float(u.sum())]
    elif expr == 2:
        coeffs = [0.3, 1.5]
    else:
        u = rng.random((n,) + interior)
        fields = (u / u.sum(axis=0)).astype(dt)
    depths = sorted({v[5] for v in V2 if v[1] == expr and v[2] == box and v[3] == r
                     and v[0] == (0 if dt == np.float32 else 1)})
    T = 23
    say("expr depths", expr, r, box, dt.__name__, depths)
    outs = []
    for bt in depths:
        plan = _plan(expr, dt, interior, r, box, T, coeffs, bt=bt)
        outs.append(_run(grid, plan, fields))
        plan.close()
    for bt, out in zip(depths[1:], outs[1:]):
        np.testing.assert_array_equal(out, outs[0], err_msg="bt=%d" % bt)
    plan = _plan(expr, dt, interior, r, box, T, coeffs)
    np.testing.assert_array_equal(_run(grid, plan, fields), outs[0])
    plan.close()
    # degenerate shapes and T = 0
    for shape, T in (((1, 1), 3), ((1, 40), 4), ((37, 2), 5), ((5, 9), 0)):
        g = rng.random(si.padded_shape(shape, r)).astype(dt)
        f = None
        if expr == 3:
            uu = rng.random((n,) + shape)
            f = (uu / uu.sum(axis=0)).astype(dt)
        plan = _plan(expr, dt, shape, r, box, T, coeffs)
        got = _run(g, plan, f)
        plan.close()
        if expr == 1:
            want = oracle.sweep_div(g.astype(np.float64), radius=r, box=box,
                                    coeffs=np.asarray(coeffs[:-1], dtype=dt).astype(np.float64),
                                    divisor=float(dt(coeffs[-1])), steps=T)
        elif expr == 2:
            want = oracle.sweep_gradient(g, cc=dt(coeffs[0]), c0=dt(coeffs[1]), steps=T)
        else:
            want = oracle.sweep_varcoef(g.astype(np.float64), radius=r, box=box,
                                        cfield=f.astype(np.float64), steps=T)
        if expr == 2 or T == 0:
            np.testing.assert_array_equal(got, want.astype(dt))
        else:
            tol = (1e-12 if dt == np.float64 else 4 * T * (n + 2) * pins.U32) * float(np.abs(want).max())
            assert float(np.max(np.abs(got.astype(np.float64) - want))) <= tol


def test_expr_plans_in_batches_and_entry_points():
    t = torch()
    rng = np.random.default_rng(801)
    interior = (150, 270)
    grid = rng.random(si.padded_shape(interior, 1))
    u = rng.random(5)
    div = _plan(1, np.float64, interior, 1, False, 17, list(u) + [float(u.sum())])
    lin = s5d.Plan(ndim=2, radius=1, box=False, dtype=np.float64, interior=interior, steps=17, coeffs=u / u.sum())
    b0 = [t.from_numpy(grid).to("cuda:0") for _ in range(2)]
    b1 = [t.empty_like(x) for x in b0]
    batch = s5d.Batch([div, lin], b0, b1)
    idx = batch.run()
    t.cuda.synchronize()
    outs = [(b0[i] if idx[i] == 0 else b1[i]).cpu().numpy() for i in range(2)]
    batch.close()
    np.testing.assert_array_equal(outs[0], _run(grid, div))
    np.testing.assert_array_equal(outs[1], _run(grid, lin))
    grad = _plan(2, np.float64, interior, 1, False, 5, [0.25, 2.0])
    x = t.from_numpy(grid).to("cuda:0")
    with pytest.raises(s5d.Stencil5DError) as err:
        s5d.Batch([grad], [x], [t.empty_like(x)])
    assert err.value.status == 2  # S5D_EUNSUPPORTED: no batched window kernel
    var = _plan(3, np.float64, interior, 1, False, 5, None)
    with pytest.raises(s5d.Stencil5DError) as err:
        var.run(x, t.empty_like(x))  # per-cell weights need s5d_run_fields
    assert err.value.status == 1
    server = s5d.Server(hbm_budget_bytes=1 << 30)
    with pytest.raises(s5d.Stencil5DError) as err:
        server.submit(grad, grid)
    assert err.value.status == 2
    server.close()
