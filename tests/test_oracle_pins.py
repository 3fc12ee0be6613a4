"""The CPU oracle against its pins (no GPU needed)."""
import numpy as np
import pytest

import oracle
import pins
import stencil_inputs as si

STENCILS_2D = [(1, False), (2, False), (3, False), (4, False), (1, True), (2, True)]
STENCILS_3D = [(1, False), (2, False), (1, True), (2, True)]


def osweep(a0, *, radius, box, coeffs, steps):
    return oracle.sweep(a0, radius=radius, box=box, coeffs=coeffs, steps=steps)


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("radius", [1, 2, 3, 4])
@pytest.mark.parametrize("box", [False, True])
def test_offsets_canonical(ndim, radius, box):
    got = oracle.offsets(ndim, radius, box)
    want = np.array(pins.canon_offsets(ndim, radius, box))
    np.testing.assert_array_equal(got, want)
    assert len(got) == si.n_points(ndim, radius, box)


def test_offsets_fig4_order():
    # the 2D 5-point star in the term order of the Fig. 4 program
    assert [tuple(o) for o in oracle.offsets(2, 1, False)] == \
        [(-1, 0), (0, -1), (0, 0), (0, 1), (1, 0)]


def test_fig4_impulse_golden():
    pins.check_fig4_impulse(osweep)


@pytest.mark.parametrize("radius,box", STENCILS_2D)
def test_dyadic_exact_2d(radius, box):
    T = pins.check_dyadic_exact(osweep, 2, radius, box, (13, 17), steps=12)
    assert T >= 6


@pytest.mark.parametrize("radius,box", STENCILS_3D)
def test_dyadic_exact_3d(radius, box):
    pins.check_dyadic_exact(osweep, 3, radius, box, (7, 6, 9), steps=6)


@pytest.mark.parametrize("ndim,radius,box", [(2, 1, False), (2, 2, True), (3, 1, True)])
def test_dyadic_exact_f32(ndim, radius, box):
    interior = (11, 9) if ndim == 2 else (5, 6, 7)
    pins.check_dyadic_exact(osweep, ndim, radius, box, interior, dtype=np.float32)


@pytest.mark.parametrize("ndim,radius,box,interior,steps", [
    (2, 1, False, (5, 6), 3), (2, 2, False, (5, 6), 2), (2, 1, True, (5, 6), 3),
    (2, 2, True, (4, 5), 2), (3, 1, False, (3, 4, 5), 2), (3, 1, True, (3, 4, 4), 2),
])
def test_rational_bound(ndim, radius, box, interior, steps):
    pins.check_rational_bound(osweep, ndim, radius, box, interior, steps)


@pytest.mark.parametrize("ndim,radius,box", [(2, r, b) for r, b in STENCILS_2D] +
                         [(3, r, b) for r, b in STENCILS_3D])
def test_single_step_scipy(ndim, radius, box):
    interior = (19, 23) if ndim == 2 else (7, 8, 9)
    pins.check_single_step_scipy(osweep, ndim, radius, box, interior)


@pytest.mark.parametrize("ndim,radius,box,steps", [
    (2, 1, False, 5), (2, 2, False, 3), (2, 4, False, 2), (2, 1, True, 4),
    (2, 2, True, 3), (3, 1, False, 3), (3, 1, True, 2), (3, 2, False, 2),
])
def test_convolution_power(ndim, radius, box, steps):
    interior = (31, 29) if ndim == 2 else (13, 12, 14)
    pins.check_convolution_power(osweep, ndim, radius, box, interior, steps)


@pytest.mark.parametrize("ndim,box,interior,modes", [
    (2, False, (21, 17), (3, 2)), (2, True, (16, 19), (1, 4)),
    (3, False, (9, 8, 11), (2, 1, 3)), (3, True, (7, 9, 8), (1, 2, 2)),
])
def test_eigenmode(ndim, box, interior, modes):
    pins.check_eigenmode(osweep, ndim, box, interior, modes, steps=25)


@pytest.mark.parametrize("ndim,radius,box", [(2, 1, False), (2, 3, False), (2, 2, True),
                                             (3, 1, False), (3, 1, True)])
def test_invariants(ndim, radius, box):
    interior = (15, 12) if ndim == 2 else (6, 7, 5)
    pins.check_constant_field(osweep, ndim, radius, box, interior, 9)
    pins.check_max_principle(osweep, ndim, radius, box, interior, 9)
    pins.check_linearity(osweep, ndim, radius, box, interior, 4)
    pins.check_composition(osweep, ndim, radius, box, interior, 5)
    pins.check_zero_steps(osweep, ndim, radius, box, interior)


@pytest.mark.parametrize("ndim,radius", [(2, 1), (2, 3), (3, 1), (3, 2)])
def test_star_is_sparse_box(ndim, radius):
    interior = (14, 11) if ndim == 2 else (6, 5, 7)
    pins.check_star_is_sparse_box(osweep, ndim, radius, interior, 4)


def test_float32_error_bound():
    """Plain float32 oracle vs float64 oracle on the same (rounded) inputs."""
    case = si.make_case(21, 2, 2, True, (40, 37), 30)
    c32, g32 = case.as_dtype(np.float32)
    r32 = oracle.sweep(g32, radius=2, box=True, coeffs=c32, steps=30)
    r64 = oracle.sweep(g32.astype(np.float64), radius=2, box=True,
                       coeffs=c32.astype(np.float64), steps=30)
    n = len(c32)
    bound = 30 * (pins.gamma(n, pins.U32) + pins.U32) * float(np.max(g32)) * 1.01
    assert float(np.max(np.abs(r32 - r64))) <= bound


def test_term_order_matches_numpy():
    """Consistency of the term order: numpy evaluates the same left-to-right sum
    (separate multiply and add, canonical order) and must give the same bits."""
    for dt in (np.float64, np.float32):
        case = si.make_case(2, 2, 2, True, (9, 10), 3)
        c, x = case.as_dtype(dt)
        offs = pins.canon_offsets(2, 2, True)
        want = x.copy()
        for _ in range(3):
            nxt = want.copy()
            acc = None
            for ck, o in zip(c, offs):
                sl = tuple(slice(2 + d, want.shape[a] - 2 + d) for a, d in enumerate(o))
                term = ck * want[sl]
                acc = term if acc is None else acc + term
            nxt[2:-2, 2:-2] = acc
            want = nxt
        got = oracle.sweep(x, radius=2, box=True, coeffs=c, steps=3)
        np.testing.assert_array_equal(got, want)


def test_rejects_bad_arguments():
    g = np.zeros((6, 6))
    with pytest.raises(ValueError):
        oracle.sweep(g, radius=1, box=False, coeffs=np.ones(4), steps=1)
    with pytest.raises(ValueError):
        oracle.sweep(g, radius=1, box=False, coeffs=np.ones(5), steps=-1)
    with pytest.raises(TypeError):
        oracle.sweep(g.astype(np.int32), radius=1, box=False, coeffs=np.ones(5), steps=1)


def test_threads_do_not_change_bits():
    case = si.make_case(30, 3, 1, True, (17, 9, 8), 4)
    a = oracle.sweep(case.grid, radius=1, box=True, coeffs=case.coeffs, steps=4, threads=1)
    b = oracle.sweep(case.grid, radius=1, box=True, coeffs=case.coeffs, steps=4, threads=4)
    np.testing.assert_array_equal(a, b)


# ---------------------------------------------------------------------------
# Compensated float32 accumulation (Dot2 of Ogita, Rump and Oishi, 2005).
# ---------------------------------------------------------------------------

def osweep_comp(a0, *, radius, box, coeffs, steps):
    return oracle.sweep(a0, radius=radius, box=box, coeffs=coeffs, steps=steps,
                        accum="compensated")


@pytest.mark.parametrize("ndim,radius,box", [(2, 1, False), (2, 2, True), (3, 1, True)])
def test_dot2_dyadic_exact(ndim, radius, box):
    interior = (13, 11) if ndim == 2 else (5, 6, 7)
    pins.check_dyadic_exact(osweep_comp, ndim, radius, box, interior, dtype=np.float32)


def _exact_step_f32(grid, radius, box, c32):
    """Exact rational value of one step's sum at every interior cell."""
    from fractions import Fraction
    nd = grid.ndim
    offs = pins.canon_offsets(nd, radius, box)
    cf = [Fraction(float(c)) for c in c32]
    out, absum = {}, {}
    inner = [idx for idx in np.ndindex(grid.shape)
             if all(radius <= idx[a] < grid.shape[a] - radius for a in range(nd))]
    for p in inner:
        s, a = Fraction(0), Fraction(0)
        for c, o in zip(cf, offs):
            x = Fraction(float(grid[tuple(p[a] + o[a] for a in range(nd))]))
            s += c * x
            a += abs(c * x)
        out[p], absum[p] = s, a
    return out, absum


@pytest.mark.parametrize("ndim,radius,box,interior", [
    (2, 1, False, (9, 10)), (2, 2, True, (7, 8)), (3, 1, True, (4, 5, 5))])
def test_dot2_single_step_bound_and_rounding(ndim, radius, box, interior):
    """|res - exact| <= u|exact| + gamma_n^2 sum|c x| per cell (the published
    bound), and res equals the correctly rounded exact sum in almost every cell."""
    case = si.make_case(61, ndim, radius, box, interior, 1)
    c32, g32 = case.as_dtype(np.float32)
    # signed coefficients make the sums ill-conditioned, where compensation matters
    rng = np.random.default_rng(3)
    c32 = (c32 * np.where(rng.random(c32.size) < 0.5, -1, 1)).astype(np.float32)
    got = oracle.sweep(g32, radius=radius, box=box, coeffs=c32, steps=1, accum="compensated")
    plain = oracle.sweep(g32, radius=radius, box=box, coeffs=c32, steps=1)
    exact, absum = _exact_step_f32(g32, radius, box, c32)
    n = len(c32)
    u = pins.U32
    g2 = pins.gamma(n, u) ** 2
    hits = plain_hits = 0
    for p, e in exact.items():
        err = abs(float(got[p]) - float(e))
        assert err <= u * abs(float(e)) + g2 * float(absum[p]) + 1e-45, (p, err)
        rn = np.float32(float(e))  # exact -> nearest float64 -> nearest float32
        hits += int(got[p] == rn)
        plain_hits += int(plain[p] == rn)
    assert hits >= 0.99 * len(exact), (hits, len(exact))
    assert hits >= plain_hits


def test_dot2_beats_plain_over_many_steps():
    case = si.make_case(62, 2, 2, True, (48, 40), 40)
    c32, g32 = case.as_dtype(np.float32)
    ref = oracle.sweep(g32.astype(np.float64), radius=2, box=True,
                       coeffs=c32.astype(np.float64), steps=40)
    comp = oracle.sweep(g32, radius=2, box=True, coeffs=c32, steps=40, accum="compensated")
    plain = oracle.sweep(g32, radius=2, box=True, coeffs=c32, steps=40)
    e_comp = np.abs(comp.astype(np.float64) - ref)
    e_plain = np.abs(plain.astype(np.float64) - ref)
    assert e_comp.max() < e_plain.max()
    assert np.sqrt(np.mean(e_comp ** 2)) < 0.5 * np.sqrt(np.mean(e_plain ** 2))
    # one float32 rounding per step at most, plus second-order terms
    assert e_comp.max() <= 40 * (pins.U32 + 25 * 25 * pins.U32 ** 2) * float(g32.max()) * 1.01


def test_dot2_rejects_float64():
    with pytest.raises(TypeError):
        oracle.sweep(np.zeros((5, 5)), radius=1, box=False, coeffs=np.ones(5), steps=1,
                     accum="compensated")
