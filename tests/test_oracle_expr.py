"""The oracle's expression and variable-coefficient sweeps against their pins
(CPU only), and planted mistakes that the pins must catch.

The expression stencils are the paper's general benchmarks (Table 3): a star
or box weighted sum divided by a constant c0 (j2d5pt -- the Fig. 4 program --,
j2d9pt, j2d9pt-gol, j3d27pt) and gradient2d; the variable-coefficient sweep
gives every cell its own weights.
"""
import numpy as np
import pytest

import oracle
import pins
import pins_expr as px

DIV_STENCILS = [(2, 1, False), (2, 2, False), (2, 1, True), (3, 1, True)]  # j2d5pt, j2d9pt, -gol, j3d27pt


def odiv(a0, *, radius, box, coeffs, divisor, steps):
    return oracle.sweep_div(a0, radius=radius, box=box, coeffs=coeffs, divisor=divisor, steps=steps)


def ograd(a0, *, cc, c0, steps):
    return oracle.sweep_gradient(a0, cc=cc, c0=c0, steps=steps)


def ovarc(a0, *, radius, box, cfield, steps):
    return oracle.sweep_varcoef(a0, radius=radius, box=box, cfield=cfield, steps=steps)


def osweep(a0, *, radius, box, coeffs, steps):
    return oracle.sweep(a0, radius=radius, box=box, coeffs=coeffs, steps=steps)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_fig4_program(dtype):
    px.check_fig4_program(odiv, dtype)


@pytest.mark.parametrize("ndim,radius,box", DIV_STENCILS)
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_div_dyadic_exact(ndim, radius, box, dtype):
    interior = (13, 17) if ndim == 2 else (6, 7, 9)
    T = px.check_div_dyadic_exact(odiv, ndim, radius, box, interior, dtype=dtype, steps=8)
    assert T >= 1


@pytest.mark.parametrize("ndim,radius,box,interior,steps", [
    (2, 1, False, (5, 6), 3), (2, 2, False, (6, 5), 2), (2, 1, True, (5, 5), 2), (3, 1, True, (3, 4, 4), 2)])
def test_div_rational_bound(ndim, radius, box, interior, steps):
    px.check_div_rational_bound(odiv, ndim, radius, box, interior, steps)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_gradient_constant_field(dtype):
    px.check_gradient_constant_field(ograd, dtype=dtype)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_gradient_ramp(dtype):
    px.check_gradient_ramp(ograd, dtype=dtype)


@pytest.mark.parametrize("dtype,steps", [(np.float64, 3), (np.float32, 2)])
def test_gradient_decimal(dtype, steps):
    px.check_gradient_decimal(ograd, steps=steps, dtype=dtype)


@pytest.mark.parametrize("ndim,radius,box", [(2, 1, False), (2, 2, True), (3, 1, False), (3, 1, True)])
def test_varcoef_uniform_and_identity(ndim, radius, box):
    interior = (9, 11) if ndim == 2 else (5, 6, 7)
    px.check_varcoef_uniform(ovarc, osweep, ndim, radius, box, interior, 4)
    px.check_varcoef_uniform(ovarc, osweep, ndim, radius, box, interior, 3, dtype=np.float32)
    px.check_varcoef_identity(ovarc, ndim, radius, box, interior)


@pytest.mark.parametrize("ndim,radius,box", [(2, 1, False), (2, 2, False), (2, 1, True), (3, 1, False)])
def test_varcoef_dyadic_exact_and_max_principle(ndim, radius, box):
    interior = (10, 13) if ndim == 2 else (5, 6, 7)
    px.check_varcoef_dyadic_exact(ovarc, ndim, radius, box, interior)
    px.check_varcoef_max_principle(ovarc, ndim, radius, box, interior)


@pytest.mark.parametrize("ndim,radius,box,interior,steps", [
    (2, 1, False, (4, 5), 3), (2, 1, True, (4, 4), 2), (3, 1, False, (3, 3, 4), 2)])
def test_varcoef_rational(ndim, radius, box, interior, steps):
    px.check_varcoef_rational(ovarc, ndim, radius, box, interior, steps)


# ---------------------------------------------------------------------------
# planted mistakes: plain numpy versions of the three sweeps with one error
# each; every mutant must fail at least one pin the oracle passes
# ---------------------------------------------------------------------------

def _np_div(a0, radius, box, coeffs, divisor, steps, *, drop=False, mul=False, mirror=False,
            divide_each=False):
    nd, r = a0.ndim, radius
    offs = pins.canon_offsets(nd, r, box)
    if mirror:
        offs = [tuple(-v for v in o) for o in offs]
    c = list(np.asarray(coeffs, dtype=a0.dtype))
    if drop:
        c, offs = c[:-1], offs[:-1]
    dv = a0.dtype.type(divisor)
    bufs = [a0.copy(), a0.copy()]
    inner = pins.interior_slices(nd, r)
    for t in range(steps):
        src, dst = bufs[t % 2], bufs[(t + 1) % 2]
        acc = None
        for ck, o in zip(c, offs):
            sl = tuple(slice(r + d, src.shape[a] - r + d) for a, d in enumerate(o))
            term = ck * src[sl]
            if divide_each:
                term = term / dv
            acc = term if acc is None else acc + term
        dst[inner] = acc if divide_each else (acc * dv if mul else acc / dv)
    return bufs[steps % 2]


def _np_grad(a0, cc, c0, steps, *, drop=False, c0_outside=False, no_square=False, diag=False):
    cc, c0 = a0.dtype.type(cc), a0.dtype.type(c0)
    nbs = [(-1, 0), (0, -1), (0, 1), (1, 0)]
    if drop:
        nbs = nbs[:-1]
    if diag:
        nbs[0] = (-1, -1)
    bufs = [a0.copy(), a0.copy()]
    for t in range(steps):
        src, dst = bufs[t % 2], bufs[(t + 1) % 2]
        f = src[1:-1, 1:-1]
        s = np.zeros_like(f) if c0_outside else np.full_like(f, c0)
        for (u, v) in nbs:
            d = f - src[1 + u:src.shape[0] - 1 + u, 1 + v:src.shape[1] - 1 + v]
            s = s + (np.abs(d) if no_square else d * d)
        root = np.sqrt(s) + c0 if c0_outside else np.sqrt(s)
        dst[1:-1, 1:-1] = cc * f + a0.dtype.type(1) / root
    return bufs[steps % 2]


def _np_varc(a0, radius, box, cfield, steps, *, transpose=False, mirror=False):
    nd, r = a0.ndim, radius
    offs = pins.canon_offsets(nd, r, box)
    cf = np.asarray(cfield, dtype=a0.dtype)
    if mirror:
        cf = cf[::-1]
    if transpose:
        cf = np.ascontiguousarray(np.swapaxes(cf, 1, 2)).reshape(cf.shape)
    bufs = [a0.copy(), a0.copy()]
    inner = pins.interior_slices(nd, r)
    for t in range(steps):
        src, dst = bufs[t % 2], bufs[(t + 1) % 2]
        acc = None
        for k, o in enumerate(offs):
            sl = tuple(slice(r + d, src.shape[a] - r + d) for a, d in enumerate(o))
            term = cf[k] * src[sl]
            acc = term if acc is None else acc + term
        dst[inner] = acc
    return bufs[steps % 2]


def _div_pins(div):
    checks = {
        "fig4": lambda: px.check_fig4_program(div),
        "dyadic": lambda: px.check_div_dyadic_exact(div, 2, 1, False, (9, 11), steps=4),
        "dyadic_box3d": lambda: px.check_div_dyadic_exact(div, 3, 1, True, (4, 5, 6), steps=2),
        "rational": lambda: px.check_div_rational_bound(div, 2, 1, False, (4, 5), 2),
    }
    return _failed(checks)


def _grad_pins(grad):
    checks = {
        "constant": lambda: px.check_gradient_constant_field(grad),
        "ramp": lambda: px.check_gradient_ramp(grad),
        "decimal": lambda: px.check_gradient_decimal(grad, steps=2),
    }
    return _failed(checks)


def _varc_pins(varc):
    checks = {
        "uniform": lambda: px.check_varcoef_uniform(varc, osweep, 2, 1, False, (7, 9), 3),
        "identity": lambda: px.check_varcoef_identity(varc, 2, 1, True, (7, 8)),
        "dyadic": lambda: px.check_varcoef_dyadic_exact(varc, 2, 1, False, (7, 9)),
        "rational": lambda: px.check_varcoef_rational(varc, 2, 1, False, (4, 5), 2),
    }
    return _failed(checks)


def _failed(checks):
    out = []
    for name, fn in checks.items():
        try:
            fn()
        except AssertionError:
            out.append(name)
    return out


DIV_MUTANTS = {"dropped_term": dict(drop=True), "multiplied": dict(mul=True),
               "mirrored_offsets": dict(mirror=True), "divides_each_term": dict(divide_each=True)}
GRAD_MUTANTS = {"dropped_neighbour": dict(drop=True), "c0_outside_root": dict(c0_outside=True),
                "no_square": dict(no_square=True), "diagonal_neighbour": dict(diag=True)}
VARC_MUTANTS = {"transposed_field": dict(transpose=True), "reversed_weights": dict(mirror=True)}


def test_mutant_baselines_pass():
    assert _div_pins(lambda a0, **k: _np_div(a0, k["radius"], k["box"], k["coeffs"], k["divisor"],
                                             k["steps"])) == []
    assert _grad_pins(lambda a0, **k: _np_grad(a0, k["cc"], k["c0"], k["steps"])) == []
    assert _varc_pins(lambda a0, **k: _np_varc(a0, k["radius"], k["box"], k["cfield"], k["steps"])) == []


@pytest.mark.parametrize("name", sorted(DIV_MUTANTS))
def test_div_mutant_caught(name):
    kw = DIV_MUTANTS[name]
    assert _div_pins(lambda a0, **k: _np_div(a0, k["radius"], k["box"], k["coeffs"], k["divisor"],
                                             k["steps"], **kw))


@pytest.mark.parametrize("name", sorted(GRAD_MUTANTS))
def test_gradient_mutant_caught(name):
    kw = GRAD_MUTANTS[name]
    assert _grad_pins(lambda a0, **k: _np_grad(a0, k["cc"], k["c0"], k["steps"], **kw))


@pytest.mark.parametrize("name", sorted(VARC_MUTANTS))
def test_varcoef_mutant_caught(name):
    kw = VARC_MUTANTS[name]
    assert _varc_pins(lambda a0, **k: _np_varc(a0, k["radius"], k["box"], k["cfield"], k["steps"], **kw))
