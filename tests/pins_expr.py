"""Independent checks ("pins") for the expression and variable-coefficient
sweeps (the paper's general benchmarks, Table 3, and per-cell weights).

Each ``check_*`` takes an implementation and raises AssertionError when it
disagrees with something the definition or plain mathematics fixes:

* the Fig. 4 program (j2d5pt: weights 5.1, 12.1, 15.0, 12.2, 5.2 and divisor
  118) applied to an impulse: its response is worked out by hand in
  tests/golden/fig4_j2d5pt_impulse.txt;
* exact dyadic arithmetic: integer weights summing to 2^q and the divisor
  2^q make every sum and quotient exact, so the result must equal an integer
  image of the sweep bit for bit;
* exact rational brute force (``fractions.Fraction``) with the a-priori
  rounding bound;
* gradient2d on fields with closed-form results: a constant field (whose
  interior follows a scalar recurrence, exact for dyadic constants) and a
  linear ramp (one step, exact for a ramp whose squared differences sum to a
  perfect square); and a 60-digit decimal brute force with a rounding bound;
* variable coefficients: uniform fields reduce to the constant-coefficient
  sweep, identity weights leave the grid unchanged, per-cell dyadic weights
  match an integer image, convex weights keep the maximum principle.

Implementations are called as
  div(a0, radius=, box=, coeffs=, divisor=, steps=)
  grad(a0, cc=, c0=, steps=)
  varc(a0, radius=, box=, cfield=, steps=)
and return A[T % 2].
"""
from __future__ import annotations

import decimal
from fractions import Fraction

import numpy as np

import pins
import stencil_inputs as si


# ---------------------------------------------------------------------------
# weighted sum / c0
# ---------------------------------------------------------------------------

def check_fig4_program(div, dtype=np.float64):
    """The Fig. 4 program on a unit impulse: the cell at displacement -o from
    the impulse receives weight(o) / 118, correctly rounded in the working
    precision; every other cell stays 0."""
    coeff, divisor, resp = pins.load_fig4()
    offs = pins.canon_offsets(2, 1, False)
    c = np.array([coeff[o] for o in offs], dtype=dtype)
    a0 = np.zeros((9, 11), dtype=dtype)
    ic = (4, 5)
    a0[ic] = 1
    got = div(a0, radius=1, box=False, coeffs=c, divisor=dtype(divisor), steps=1)
    expect = np.zeros_like(a0)
    for (d0, d1), val in resp:
        a, b = (int(v) for v in val[len("coeff"):].strip("()").split(","))
        expect[ic[0] + d0, ic[1] + d1] = dtype(coeff[(a, b)]) / dtype(divisor)
    np.testing.assert_array_equal(got, expect)
    # two impulses two rows apart: one cell adds two products, then divides
    at, (oa, ob) = pins.load_fig4_pair()
    a0[ic[0] + 2, ic[1]] = 1
    got = div(a0, radius=1, box=False, coeffs=c, divisor=dtype(divisor), steps=1)
    want = (dtype(coeff[oa]) + dtype(coeff[ob])) / dtype(divisor)
    assert got[ic[0] + at[0], ic[1] + at[1]] == want


def _dyadic_div_case(ndim, radius, box, interior, seed):
    case = si.make_dyadic_case(seed, ndim, radius, box, interior, 1)
    return case


def check_div_dyadic_exact(div, ndim, radius, box, interior, dtype=np.float64, seed=21, steps=None):
    """Integer weights w_k (summing to 2^q) with divisor 2^q: exact."""
    bits = 53 if np.dtype(dtype) == np.float64 else 24
    case = _dyadic_div_case(ndim, radius, box, interior, seed)
    q, m = case.meta["q"], case.meta["m"]
    tmax = si.max_exact_steps(q, m, bits)
    T = tmax if steps is None else min(steps, tmax)
    case.steps = T
    ints, e = pins.exact_integer_sweep(case)
    w = np.asarray(case.meta["weights"], dtype=dtype)
    got = div(case.grid.astype(dtype), radius=radius, box=box, coeffs=w,
              divisor=dtype(2.0 ** q), steps=T)
    want = np.ldexp(ints.astype(np.float64), -e).astype(dtype)
    np.testing.assert_array_equal(got, want)
    return T


def check_div_rational_bound(div, ndim, radius, box, interior, steps, seed=22):
    """Random weights and divisor: within T * gamma_{n+1} of the exact
    rational result (the operator's infinity norm is sum|c|/c0 < 1 here)."""
    rng = np.random.default_rng(seed)
    n = si.n_points(ndim, radius, box)
    c = rng.random(n)
    c0 = float(c.sum() * (1.0 + rng.random()))
    grid = rng.random(si.padded_shape(interior, radius))
    # exact rational sweep with the divisor applied to every step's sum
    offs = pins.canon_offsets(ndim, radius, box)
    cf = [Fraction(float(v)) for v in c]
    d = Fraction(c0)
    cur = {idx: Fraction(float(v)) for idx, v in np.ndenumerate(grid)}
    shape = grid.shape
    inner = [idx for idx in cur if all(radius <= idx[a] < shape[a] - radius for a in range(ndim))]
    for _ in range(steps):
        nxt = dict(cur)
        for p in inner:
            s = Fraction(0)
            for ck, o in zip(cf, offs):
                s += ck * cur[tuple(p[a] + o[a] for a in range(ndim))]
            nxt[p] = s / d
        cur = nxt
    got = div(grid, radius=radius, box=box, coeffs=c, divisor=c0, steps=steps)
    err = max(abs(Fraction(float(got[idx])) - v) for idx, v in cur.items())
    bound = steps * pins.gamma(n + 1, pins.U64) * float(grid.max())
    assert float(err) <= bound * 1.01, (float(err), bound)


# ---------------------------------------------------------------------------
# gradient2d
# ---------------------------------------------------------------------------

def check_gradient_constant_field(grad, interior=(13, 15), steps=5, dtype=np.float64):
    """f = a everywhere (boundary included): after t steps an interior cell
    whose distance to the boundary exceeds t still sees equal neighbours, so
    it follows f_{t+1} = cc f_t + 1/sqrt(c0); with a = 1/2, cc = 1/4 and
    c0 = 4 every value is dyadic and exact."""
    a, cc, c0 = Fraction(1, 2), Fraction(1, 4), Fraction(4)
    grid = np.full(si.padded_shape(interior, 1), float(a), dtype=dtype)
    got = grad(grid, cc=dtype(cc), c0=dtype(c0), steps=steps)
    f = a
    for _ in range(steps):
        f = cc * f + Fraction(1, 2)  # 1/sqrt(4)
    inner = got[1 + steps:-1 - steps, 1 + steps:-1 - steps]
    assert inner.size > 0
    np.testing.assert_array_equal(inner, np.full(inner.shape, float(f), dtype=dtype))
    # the boundary never changes
    np.testing.assert_array_equal(got[0, :], grid[0, :])
    np.testing.assert_array_equal(got[:, -1], grid[:, -1])


def check_gradient_ramp(grad, interior=(9, 12), dtype=np.float64):
    """f(i, j) = (i + j) / 4 on the whole padded grid: every interior cell
    has squared differences 1/16 four times, so with c0 = 3/4 the root is 1
    and one step gives cc f + 1 exactly."""
    P = si.padded_shape(interior, 1)
    i, j = np.meshgrid(np.arange(P[0]), np.arange(P[1]), indexing="ij")
    grid = ((i + j) / 4.0).astype(dtype)
    cc = dtype(0.375)
    got = grad(grid, cc=cc, c0=dtype(0.75), steps=1)
    want = grid.copy()
    want[1:-1, 1:-1] = cc * grid[1:-1, 1:-1] + dtype(1)
    np.testing.assert_array_equal(got, want)


def _decimal_gradient(grid, cc, c0, steps, digits=60):
    ctx = decimal.Context(prec=digits)
    D = lambda v: ctx.create_decimal_from_float(float(v))  # noqa: E731
    cur = [[D(v) for v in row] for row in grid]
    dcc, dc0 = D(cc), D(c0)
    P0, P1 = grid.shape
    for _ in range(steps):
        nxt = [row[:] for row in cur]
        for a in range(1, P0 - 1):
            for b in range(1, P1 - 1):
                f = cur[a][b]
                s = dc0
                for (u, v) in ((a - 1, b), (a, b - 1), (a, b + 1), (a + 1, b)):
                    d = ctx.subtract(f, cur[u][v])
                    s = ctx.add(s, ctx.multiply(d, d))
                nxt[a][b] = ctx.add(ctx.multiply(dcc, f), ctx.divide(1, ctx.sqrt(s)))
        cur = nxt
    return cur


def check_gradient_decimal(grad, interior=(5, 7), steps=3, seed=24, dtype=np.float64):
    """Against a 60-digit decimal evaluation of the same recurrence: each step
    rounds 15 operations per cell, and the map's sensitivity to its inputs is
    bounded by cc + 8 max|d| / c0^(3/2) <= 2.5 here (c0 >= 1, |d| < 1/8 after
    scaling), so the error stays within 16 * 15 u * 2.5^T * max|f|."""
    rng = np.random.default_rng(seed)
    grid = (rng.random(si.padded_shape(interior, 1)) / 8.0).astype(dtype)
    cc = dtype(rng.random() / 2)
    c0 = dtype(1.0 + rng.random())
    got = grad(grid, cc=cc, c0=c0, steps=steps)
    ref = _decimal_gradient(grid, cc, c0, steps)
    u = pins.U64 if np.dtype(dtype) == np.float64 else pins.U32
    err = max(abs(decimal.Decimal(float(got[a, b])) - ref[a][b])
              for a in range(grid.shape[0]) for b in range(grid.shape[1]))
    mag = max(abs(v) for row in ref for v in row)
    bound = 16 * 15 * u * (2.5 ** steps) * float(mag)
    assert float(err) <= bound, (float(err), bound)


# ---------------------------------------------------------------------------
# variable coefficients
# ---------------------------------------------------------------------------

def check_varcoef_uniform(varc, sweep, ndim, radius, box, interior, steps, seed=25, dtype=np.float64):
    """Uniform weight fields reduce to the constant-coefficient sweep: the same
    products and sums in the same order, so the same bits."""
    rng = np.random.default_rng(seed)
    n = si.n_points(ndim, radius, box)
    c = si.random_coeffs(rng, n).astype(dtype)
    grid = rng.random(si.padded_shape(interior, radius)).astype(dtype)
    cf = np.empty((n,) + tuple(interior), dtype=dtype)
    for k in range(n):
        cf[k] = c[k]
    got = varc(grid, radius=radius, box=box, cfield=cf, steps=steps)
    want = sweep(grid, radius=radius, box=box, coeffs=c, steps=steps)
    np.testing.assert_array_equal(got, want)


def check_varcoef_identity(varc, ndim, radius, box, interior, steps=3, seed=26):
    rng = np.random.default_rng(seed)
    offs = pins.canon_offsets(ndim, radius, box)
    n = len(offs)
    cf = np.zeros((n,) + tuple(interior))
    cf[offs.index((0,) * ndim)] = 1.0
    grid = rng.random(si.padded_shape(interior, radius))
    np.testing.assert_array_equal(varc(grid, radius=radius, box=box, cfield=cf, steps=steps), grid)


def check_varcoef_dyadic_exact(varc, ndim, radius, box, interior, steps=4, seed=27, q=6, m=4):
    """Per-cell integer weights summing to 2^q, grid m/2^m: every product and
    sum is exact for T steps while m + qT <= 53, so the result equals integer
    arithmetic on the scaled values."""
    rng = np.random.default_rng(seed)
    offs = pins.canon_offsets(ndim, radius, box)
    n = len(offs)
    assert m + q * steps <= 53
    # random compositions of 2^q into n non-negative parts, one per cell
    cuts = np.sort(rng.integers(0, 2 ** q + 1, size=(n - 1,) + tuple(interior)), axis=0)
    lo = np.concatenate([np.zeros((1,) + tuple(interior), dtype=np.int64), cuts], axis=0)
    hi = np.concatenate([cuts, np.full((1,) + tuple(interior), 2 ** q, dtype=np.int64)], axis=0)
    w = hi - lo
    assert np.all(w.sum(axis=0) == 2 ** q)
    x = rng.integers(0, 2 ** m, size=si.padded_shape(interior, radius)).astype(np.int64)
    grid = np.ldexp(x.astype(np.float64), -m)
    inner = pins.interior_slices(ndim, radius)
    for _ in range(steps):
        y = x << q
        acc = np.zeros_like(x[inner])
        for k, o in enumerate(offs):
            sl = tuple(slice(radius + d, x.shape[a] - radius + d) for a, d in enumerate(o))
            acc += w[k] * x[sl]
        y[inner] = acc
        x = y
    want = np.ldexp(x.astype(np.float64), -(m + q * steps))
    got = varc(grid, radius=radius, box=box, cfield=np.ldexp(w.astype(np.float64), -q), steps=steps)
    np.testing.assert_array_equal(got, want)


def check_varcoef_max_principle(varc, ndim, radius, box, interior, steps=6, seed=28):
    """Convex per-cell weights keep every value within [min A0, max A0]."""
    rng = np.random.default_rng(seed)
    n = si.n_points(ndim, radius, box)
    u = rng.random((n,) + tuple(interior))
    cf = u / u.sum(axis=0)
    grid = rng.random(si.padded_shape(interior, radius))
    got = varc(grid, radius=radius, box=box, cfield=cf, steps=steps)
    slack = steps * pins.gamma(n, pins.U64) * float(grid.max()) * 1.01
    assert got.min() >= grid.min() - slack and got.max() <= grid.max() + slack
    # and it is not the identity
    assert np.any(got != grid)


def check_varcoef_rational(varc, ndim, radius, box, interior, steps, seed=29):
    """Exact rational brute force: the per-cell linear map applied T times,
    within T * gamma_n of the float64 result (convex weights)."""
    rng = np.random.default_rng(seed)
    offs = pins.canon_offsets(ndim, radius, box)
    n = len(offs)
    u = rng.random((n,) + tuple(interior))
    cf = u / u.sum(axis=0)
    grid = rng.random(si.padded_shape(interior, radius))
    cur = {idx: Fraction(float(v)) for idx, v in np.ndenumerate(grid)}
    for _ in range(steps):
        nxt = dict(cur)
        for q in np.ndindex(*interior):
            p = tuple(q[a] + radius for a in range(ndim))
            s = Fraction(0)
            for k, o in enumerate(offs):
                s += Fraction(float(cf[(k,) + q])) * cur[tuple(p[a] + o[a] for a in range(ndim))]
            nxt[p] = s
        cur = nxt
    got = varc(grid, radius=radius, box=box, cfield=cf, steps=steps)
    err = max(abs(Fraction(float(got[idx])) - v) for idx, v in cur.items())
    bound = steps * pins.gamma(n, pins.U64) * float(grid.max()) * 1.01
    assert float(err) <= bound, (float(err), bound)
