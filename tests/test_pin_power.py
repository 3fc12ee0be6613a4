"""The pins catch plausible mistakes.

Each mutant below is a deliberately wrong sweep (a dropped term, mirrored
offsets, swapped axes, a boundary that gets updated, the wrong result buffer,
a transposed box coefficient order, float32 accumulation, one extra step).
Every mutant must fail at least one of the pins the oracle passes, which shows
the pins would have caught that mistake in the oracle.  Everything runs on the
CPU.
"""
import numpy as np
import pytest

import pins


def _reference_sweep(a0, radius, box, coeffs, steps, *, offs_fn=None, drop=False,
                     update_halo=False, wrong_parity=False, acc32=False, extra=0):
    nd = a0.ndim
    offs = (offs_fn or pins.canon_offsets)(nd, radius, box)
    c = list(np.asarray(coeffs, dtype=np.float64))
    if drop:
        c, offs = c[:-1], offs[:-1]
    r = radius
    bufs = [np.array(a0, dtype=np.float64), np.array(a0, dtype=np.float64)]
    inner = tuple(slice(r, s - r) for s in a0.shape)
    for t in range(steps + extra):
        src, dst = bufs[t % 2], bufs[(t + 1) % 2]
        acc = None
        for ck, o in zip(c, offs):
            sl = tuple(slice(r + d, src.shape[a] - r + d) for a, d in enumerate(o))
            term = ck * src[sl]
            if acc32:
                term = term.astype(np.float32)
            acc = term if acc is None else acc + term
        dst[inner] = acc
        if update_halo:
            dst[tuple(slice(0, 1) for _ in range(nd))] += 1.0
    idx = (steps + extra + (1 if wrong_parity else 0)) % 2
    return bufs[idx].astype(a0.dtype)


def _mirrored(nd, r, box):
    return [tuple(-v for v in o) for o in pins.canon_offsets(nd, r, box)]


def _swapped(nd, r, box):
    return [tuple(reversed(o)) for o in pins.canon_offsets(nd, r, box)]


MUTANTS = {
    "dropped_term": dict(drop=True),
    "mirrored_offsets": dict(offs_fn=_mirrored),
    "swapped_axes": dict(offs_fn=_swapped),
    "boundary_written": dict(update_halo=True),
    "wrong_result_buffer": dict(wrong_parity=True),
    "float32_accumulation": dict(acc32=True),
    "one_extra_step": dict(extra=1),
}


def _mutant(kw):
    def sweep(a0, *, radius, box, coeffs, steps):
        return _reference_sweep(a0, radius, box, coeffs, steps, **kw)
    return sweep


def _all_pins(sweep):
    """Run a representative subset of the pins; return the names that fail."""
    checks = {
        "fig4": lambda: pins.check_fig4_impulse(sweep),
        "dyadic": lambda: pins.check_dyadic_exact(sweep, 2, 1, False, (9, 11), steps=5),
        "dyadic_box": lambda: pins.check_dyadic_exact(sweep, 2, 1, True, (9, 11), steps=5),
        "scipy1": lambda: pins.check_single_step_scipy(sweep, 2, 2, True, (11, 13)),
        "convpow": lambda: pins.check_convolution_power(sweep, 2, 1, True, (15, 16), 3),
        "eigen": lambda: pins.check_eigenmode(sweep, 2, False, (13, 11), (2, 3), 6),
        "rational": lambda: pins.check_rational_bound(sweep, 2, 1, False, (4, 5), 2),
        "composition": lambda: pins.check_composition(sweep, 2, 1, False, (8, 7), 3),
        "linearity": lambda: pins.check_linearity(sweep, 2, 1, False, (8, 9), 3),
    }
    failed = []
    for name, fn in checks.items():
        try:
            fn()
        except AssertionError:
            failed.append(name)
    return failed


def test_reference_mutant_baseline_passes():
    """The unmutated numpy sweep passes every pin (so failures below are real)."""
    assert _all_pins(_mutant({})) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name):
    failed = _all_pins(_mutant(MUTANTS[name]))
    assert failed, "mutant %s passed every pin" % name
