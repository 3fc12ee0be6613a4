"""Independent checks ("pins") for any implementation of the stencil sweep.

Each ``check_*`` takes a ``sweep(a0, radius=, box=, coeffs=, steps=)`` callable
that returns A[T % 2] for the padded initial grid ``a0`` and raises
AssertionError when the implementation disagrees with something the paper's
definition or plain mathematics fixes:

* exact dyadic arithmetic (integer numpy arithmetic, no floating point),
* exact rational brute force (``fractions.Fraction``) with Higham's bound,
* scipy's direct correlate / convolve (single step and convolution power),
* closed-form sine eigenmodes,
* the maximum principle, preservation of a constant field, linearity,
* composition of single steps, and
* a hand-derived impulse response for the coefficients printed in Fig. 4.

The offsets are enumerated here on their own (itertools), not taken from the
implementation under test.
"""
from __future__ import annotations

import itertools
import math
import os
from fractions import Fraction

import numpy as np
import scipy.signal

import stencil_inputs as si

U64 = 2.0 ** -53
U32 = 2.0 ** -24
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def canon_offsets(ndim, radius, box):
    """Lexicographic (d0, d1[, d2]) offsets, axis 0 slowest; star keeps axis lines."""
    rng = range(-radius, radius + 1)
    out = []
    for o in itertools.product(rng, repeat=ndim):
        if box or sum(1 for v in o if v != 0) <= 1:
            out.append(o)
    return out


def dense_kernel(ndim, radius, box, coeffs):
    """(2r+1)^d array K with K[o + r] = c_k for canonical offset k."""
    K = np.zeros((2 * radius + 1,) * ndim)
    for c, o in zip(coeffs, canon_offsets(ndim, radius, box)):
        K[tuple(v + radius for v in o)] = c
    return K


def gamma(n, u):
    return n * u / (1.0 - n * u)


def interior_slices(ndim, radius):
    return tuple(slice(radius, -radius) for _ in range(ndim))


# ---------------------------------------------------------------------------
# P1: exact dyadic arithmetic, checked against integer arithmetic.
# ---------------------------------------------------------------------------

def exact_integer_sweep(case):
    """Integer image of the sweep on dyadic inputs.

    Values are held as integers scaled by 2**(m + q*t).  One step multiplies
    the scale by 2**q: interior cells become sum_k w_k * x[p + o_k] and the
    fixed boundary cells are rescaled by 2**q.  Returns (ints, scale_exp).
    """
    q, m = case.meta["q"], case.meta["m"]
    w = case.meta["weights"]
    x = case.meta["grid_ints"].astype(np.int64)
    r, nd = case.radius, case.ndim
    offs = canon_offsets(nd, r, case.box)
    inner = interior_slices(nd, r)
    for _ in range(case.steps):
        y = x << q
        acc = np.zeros_like(x[inner])
        for wk, o in zip(w, offs):
            sl = tuple(slice(r + d, x.shape[a] - r + d) for a, d in enumerate(o))
            acc += int(wk) * x[sl]
        y[inner] = acc
        x = y
    return x, m + q * case.steps


def check_dyadic_exact(sweep, ndim, radius, box, interior, dtype=np.float64, seed=11,
                       steps=None):
    bits = 53 if np.dtype(dtype) == np.float64 else 24
    case = si.make_dyadic_case(seed, ndim, radius, box, interior, 1)
    q, m = case.meta["q"], case.meta["m"]
    tmax = si.max_exact_steps(q, m, bits)
    T = tmax if steps is None else min(steps, tmax)
    assert T >= 1
    case.steps = T
    ints, e = exact_integer_sweep(case)
    got = sweep(case.grid.astype(dtype), radius=radius, box=box,
                coeffs=case.coeffs.astype(dtype), steps=T)
    want = np.ldexp(ints.astype(np.float64), -e).astype(dtype)
    np.testing.assert_array_equal(got, want)
    return T


# ---------------------------------------------------------------------------
# P2: exact rational brute force with the a-priori rounding bound.
# ---------------------------------------------------------------------------

def rational_sweep(grid, radius, box, coeffs, steps):
    """Fraction arithmetic on the exact binary values of the float inputs."""
    nd = grid.ndim
    offs = canon_offsets(nd, radius, box)
    cf = [Fraction(float(c)) for c in coeffs]
    cur = {idx: Fraction(float(v)) for idx, v in np.ndenumerate(grid)}
    shape = grid.shape
    inner = [idx for idx in cur if all(radius <= idx[a] < shape[a] - radius
                                       for a in range(nd))]
    for _ in range(steps):
        nxt = dict(cur)
        for p in inner:
            s = Fraction(0)
            for c, o in zip(cf, offs):
                s += c * cur[tuple(p[a] + o[a] for a in range(nd))]
            nxt[p] = s
        cur = nxt
    out = np.empty(shape, dtype=object)
    for idx, v in cur.items():
        out[idx] = v
    return out


def check_rational_bound(sweep, ndim, radius, box, interior, steps, seed=5):
    case = si.make_case(seed, ndim, radius, box, interior, steps)
    exact = rational_sweep(case.grid, radius, box, case.coeffs, steps)
    got = sweep(case.grid, radius=radius, box=box, coeffs=case.coeffs, steps=steps)
    n = len(case.coeffs)
    M = float(np.max(np.abs(case.grid)))
    s1 = float(sum(Fraction(float(c)) for c in case.coeffs))  # sum |c| (all c >= 0)
    bound = steps * gamma(n, U64) * M * max(1.0, s1) ** steps * 1.01
    err = max(abs(Fraction(float(g)) - e) for g, e in zip(got.ravel(), exact.ravel()))
    assert float(err) <= bound, "error %g exceeds bound %g" % (float(err), bound)
    return float(err), bound


# ---------------------------------------------------------------------------
# P8 / P7: scipy direct correlate, one step and the convolution power.
# ---------------------------------------------------------------------------

def check_single_step_scipy(sweep, ndim, radius, box, interior, seed=3):
    case = si.make_case(seed, ndim, radius, box, interior, 1)
    got = sweep(case.grid, radius=radius, box=box, coeffs=case.coeffs, steps=1)
    K = dense_kernel(ndim, radius, box, case.coeffs)
    want = scipy.signal.correlate(case.grid, K, mode="valid", method="direct")
    inner = interior_slices(ndim, radius)
    n = K.size
    tol = 4 * n * U64 * float(np.max(np.abs(case.grid)))
    assert np.max(np.abs(got[inner] - want)) <= tol
    # the fixed boundary is carried through untouched
    mask = np.ones(case.grid.shape, bool)
    mask[inner] = False
    np.testing.assert_array_equal(got[mask], case.grid[mask])


def check_convolution_power(sweep, ndim, radius, box, interior, steps, seed=4):
    case = si.make_case(seed, ndim, radius, box, interior, steps)
    got = sweep(case.grid, radius=radius, box=box, coeffs=case.coeffs, steps=steps)
    K = dense_kernel(ndim, radius, box, case.coeffs)
    KT = K
    for _ in range(steps - 1):
        KT = scipy.signal.convolve(KT, K, mode="full", method="direct")
    want = scipy.signal.correlate(case.grid, KT, mode="valid", method="direct")
    lo = steps * radius
    sl = tuple(slice(lo, lo + want.shape[a]) for a in range(ndim))
    tol = 4 * (steps * K.size + KT.size) * U64 * float(np.max(np.abs(case.grid)))
    err = float(np.max(np.abs(got[sl] - want)))
    assert err <= tol, "error %g > %g" % (err, tol)


# ---------------------------------------------------------------------------
# P6: closed-form sine eigenmodes with a zero boundary (radius 1).
# ---------------------------------------------------------------------------

def eigen_case(ndim, box, interior, modes, seed=9):
    rng = np.random.default_rng(seed)
    shape = tuple(i + 2 for i in interior)
    thetas = [p * math.pi / (I + 1) for p, I in zip(modes, interior)]
    grids = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    u = np.ones(shape)
    for g, th in zip(grids, thetas):
        u = u * np.sin(th * g)
    inner = interior_slices(ndim, 1)
    u0 = np.zeros(shape)
    u0[inner] = u[inner]
    if box:
        # tensor product of symmetric 1D weights (a0, a1, a0... per axis)
        axw = []
        for _ in range(ndim):
            a1 = rng.uniform(0.05, 0.3)
            axw.append((a1, 1.0 - 2 * a1))
        offs = canon_offsets(ndim, 1, True)
        coeffs = np.array([np.prod([axw[a][0] if o[a] != 0 else axw[a][1]
                                    for a in range(ndim)]) for o in offs])
        lam = np.prod([w0 + 2 * w1 * math.cos(th) for (w1, w0), th in zip(axw, thetas)])
    else:
        side = rng.uniform(0.05, 0.15, size=ndim)  # one weight per axis, both sides
        c0 = 1.0 - 2 * side.sum()
        offs = canon_offsets(ndim, 1, False)
        coeffs = []
        for o in offs:
            nz = [a for a in range(ndim) if o[a] != 0]
            coeffs.append(c0 if not nz else side[nz[0]])
        coeffs = np.array(coeffs)
        lam = c0 + sum(2 * side[a] * math.cos(thetas[a]) for a in range(ndim))
    return u0, coeffs, lam


def check_eigenmode(sweep, ndim, box, interior, modes, steps):
    u0, coeffs, lam = eigen_case(ndim, box, interior, modes)
    got = sweep(u0, radius=1, box=box, coeffs=coeffs, steps=steps)
    want = (lam ** steps) * u0
    tol = 8 * steps * len(coeffs) * U64
    err = float(np.max(np.abs(got - want)))
    assert err <= tol, "eigenmode error %g > %g" % (err, tol)


# ---------------------------------------------------------------------------
# Invariants.
# ---------------------------------------------------------------------------

def check_constant_field(sweep, ndim, radius, box, interior, steps, seed=6):
    shape = si.padded_shape(interior, radius)
    val = 0.8125
    n = si.n_points(ndim, radius, box)
    dy = si.make_dyadic_case(seed, ndim, radius, box, interior, 1)
    got = sweep(np.full(shape, val), radius=radius, box=box, coeffs=dy.coeffs, steps=steps)
    np.testing.assert_array_equal(got, np.full(shape, val))
    c = si.random_coeffs(np.random.default_rng(seed), n)
    got = sweep(np.full(shape, val), radius=radius, box=box, coeffs=c, steps=steps)
    drift = abs(float(np.sum(c)) - 1.0) * steps
    tol = (steps * gamma(n, U64) + drift) * val * 1.01
    assert float(np.max(np.abs(got - val))) <= tol


def check_max_principle(sweep, ndim, radius, box, interior, steps, seed=7):
    case = si.make_case(seed, ndim, radius, box, interior, steps)
    got = sweep(case.grid, radius=radius, box=box, coeffs=case.coeffs, steps=steps)
    lo, hi = float(case.grid.min()), float(case.grid.max())
    slack = steps * gamma(len(case.coeffs), U64) * hi * 1.01
    assert got.min() >= lo - slack and got.max() <= hi + slack


def check_linearity(sweep, ndim, radius, box, interior, steps, seed=8):
    """S(a u + b v) == a S(u) + b S(v), bit for bit on dyadic data."""
    cu = si.make_dyadic_case(seed, ndim, radius, box, interior, steps, m=3)
    cv = si.make_dyadic_case(seed + 1, ndim, radius, box, interior, steps, m=3)
    c = cu.coeffs
    a, b = 0.5, 0.25
    su = sweep(cu.grid, radius=radius, box=box, coeffs=c, steps=steps)
    sv = sweep(cv.grid, radius=radius, box=box, coeffs=c, steps=steps)
    sw = sweep(a * cu.grid + b * cv.grid, radius=radius, box=box, coeffs=c, steps=steps)
    np.testing.assert_array_equal(sw, a * su + b * sv)


def check_composition(sweep, ndim, radius, box, interior, steps, seed=10):
    case = si.make_case(seed, ndim, radius, box, interior, steps)
    full = sweep(case.grid, radius=radius, box=box, coeffs=case.coeffs, steps=steps)
    x = case.grid
    for _ in range(steps):
        x = sweep(x, radius=radius, box=box, coeffs=case.coeffs, steps=1)
    np.testing.assert_array_equal(full, x)


def check_zero_steps(sweep, ndim, radius, box, interior, seed=12):
    case = si.make_case(seed, ndim, radius, box, interior, 0)
    got = sweep(case.grid, radius=radius, box=box, coeffs=case.coeffs, steps=0)
    np.testing.assert_array_equal(got, case.grid)


def check_star_is_sparse_box(sweep, ndim, radius, interior, steps, seed=13):
    """A star equals the box whose off-axis coefficients are zero (bit for bit)."""
    case = si.make_case(seed, ndim, radius, False, interior, steps)
    K = dense_kernel(ndim, radius, False, case.coeffs)
    cbox = np.array([K[tuple(v + radius for v in o)]
                     for o in canon_offsets(ndim, radius, True)])
    s = sweep(case.grid, radius=radius, box=False, coeffs=case.coeffs, steps=steps)
    b = sweep(case.grid, radius=radius, box=True, coeffs=cbox, steps=steps)
    np.testing.assert_array_equal(s, b)


# ---------------------------------------------------------------------------
# Golden: the Fig. 4 coefficients, impulse response worked out by hand.
# ---------------------------------------------------------------------------

def load_fig4():
    """Parse tests/golden/fig4_j2d5pt_impulse.txt."""
    path = os.path.join(GOLDEN, "fig4_j2d5pt_impulse.txt")
    coeff, resp = {}, []
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            key, _, val = line.partition("=")
            key, val = key.strip(), val.strip()
            if key == "divisor":
                div = float(val)
            elif key.startswith("coeff"):
                d0, d1 = (int(v) for v in key[len("coeff"):].strip("()").split(","))
                coeff[(d0, d1)] = float(val)
            elif key.startswith("response"):
                d0, d1 = (int(v) for v in key[len("response"):].strip("()").split(","))
                resp.append(((d0, d1), val))
    return coeff, div, resp


def load_fig4_pair():
    """The second worked example of the Fig. 4 golden file: the displacement
    of the cell that sums two non-zero products, and the two offsets whose
    weights it adds (in the program's order) before dividing."""
    path = os.path.join(GOLDEN, "fig4_j2d5pt_impulse.txt")
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line.startswith("pair"):
                key, _, val = line.partition("=")
                at = tuple(int(v) for v in key[len("pair"):].strip(" ()").split(","))
                terms = val.split("/")[0].strip(" ()").split("+")
                offs = [tuple(int(v) for v in t.strip()[len("coeff"):].strip("()").split(","))
                        for t in terms]
                return at, offs
    raise ValueError("no pair line in the Fig. 4 golden file")


def check_fig4_impulse(sweep):
    coeff, div, resp = load_fig4()
    offs = canon_offsets(2, 1, False)
    c = np.array([coeff[o] / div for o in offs])
    a0 = np.zeros((9, 9))
    ic = (4, 4)
    a0[ic] = 1.0
    got = sweep(a0, radius=1, box=False, coeffs=c, steps=1)
    named = {o: coeff[o] / div for o in coeff}
    expect = np.zeros_like(a0)
    for (d0, d1), val in resp:
        # the value is written as "coeff(a,b)": the weight that lands there
        a, b = (int(v) for v in val[len("coeff"):].strip("()").split(","))
        expect[ic[0] + d0, ic[1] + d1] = named[(a, b)]
    np.testing.assert_array_equal(got, expect)
