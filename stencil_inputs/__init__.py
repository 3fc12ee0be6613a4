"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no stencil arithmetic: it only draws coefficients and
padded grids from seeded generators, so that the CPU oracle and the GPU
library can be fed the very same numbers.  Neither of those imports the other;
both may be fed from here.

Recipe (the paper evaluates synthetic star/box stencils on 16384^2 and 512^3
grids, Table 3 and "Methodology"; no dataset is involved):

* generator: numpy PCG64, ``np.random.default_rng(seed)``;
* coefficients: ``u = rng.random(n)``, ``c = u / u.sum()`` in float64, so they
  are positive and sum to one (up to rounding);
* grid: ``rng.random(padded_shape)`` in C order, boundary cells included,
  float64; float32 runs cast both with round-to-nearest;
* seeds: base 1473; workload i uses ``1473 + i``; item j of a batch or serving
  mix uses ``seed * 10**6 + j``.

The dyadic generators produce inputs on which every product and partial sum
of a sweep is exact in binary floating point (coefficients are multiples of
2**-q summing to exactly 1, grid values are multiples of 2**-m), so any
correct implementation must return the same bits regardless of term order,
fused multiply-add or temporal blocking.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 1473


def workload_seed(i: int) -> int:
    return BASE_SEED + i


def item_seed(seed: int, j: int) -> int:
    return seed * 10**6 + j


def n_points(ndim: int, radius: int, box: bool) -> int:
    """Number of stencil points: star 2*r*d + 1, box (2r+1)**d."""
    return (2 * radius + 1) ** ndim if box else 2 * radius * ndim + 1


def padded_shape(interior, radius: int):
    return tuple(int(i) + 2 * radius for i in interior)


def random_coeffs(rng: np.random.Generator, n: int) -> np.ndarray:
    u = rng.random(n)
    return u / u.sum()


def random_grid(rng: np.random.Generator, shape) -> np.ndarray:
    return rng.random(tuple(shape))


@dataclass
class Case:
    """One stencil problem: descriptor fields plus its seeded inputs (float64)."""
    ndim: int
    radius: int
    box: bool
    interior: tuple
    steps: int
    coeffs: np.ndarray
    grid: np.ndarray
    seed: int = 0
    meta: dict = field(default_factory=dict)

    def as_dtype(self, dtype):
        """Coefficients and grid rounded to ``dtype`` (round to nearest)."""
        dt = np.dtype(dtype)
        return self.coeffs.astype(dt), self.grid.astype(dt)


def make_case(seed: int, ndim: int, radius: int, box: bool, interior, steps: int) -> Case:
    """Random coefficients then a random padded grid, both from one PCG64 stream."""
    interior = tuple(int(i) for i in interior)
    if len(interior) != ndim:
        raise ValueError("interior must have ndim entries")
    rng = np.random.default_rng(seed)
    c = random_coeffs(rng, n_points(ndim, radius, box))
    g = random_grid(rng, padded_shape(interior, radius))
    return Case(ndim, radius, box, interior, int(steps), c, g, seed)


def dyadic_weights(rng: np.random.Generator, n: int, q: int) -> np.ndarray:
    """n positive integers summing to exactly 2**q (needs 2**q >= n)."""
    total = 1 << q
    if total < n:
        raise ValueError("2**q must be at least n")
    extra = rng.multinomial(total - n, np.full(n, 1.0 / n))
    return (1 + extra).astype(np.int64)


def min_dyadic_q(n: int) -> int:
    return max(1, math.ceil(math.log2(n)))


def make_dyadic_case(seed: int, ndim: int, radius: int, box: bool, interior, steps: int,
                     q: int | None = None, m: int = 4) -> Case:
    """Exactly representable inputs: c_k = w_k / 2**q (sum 1), grid = k / 2**m.

    After t steps every value is a multiple of 2**-(m + q*t) in [0, 1), so a
    sweep of T steps is exact in a binary format with p mantissa bits while
    m + q*T <= p (53 for float64, 24 for float32).
    """
    interior = tuple(int(i) for i in interior)
    n = n_points(ndim, radius, box)
    q = min_dyadic_q(n) if q is None else q
    rng = np.random.default_rng(seed)
    w = dyadic_weights(rng, n, q)
    c = w.astype(np.float64) / float(1 << q)
    k = rng.integers(0, 1 << m, size=padded_shape(interior, radius))
    g = k.astype(np.float64) / float(1 << m)
    case = Case(ndim, radius, box, interior, int(steps), c, g, seed)
    case.meta.update(q=q, m=m, weights=w, grid_ints=k)
    return case


def max_exact_steps(q: int, m: int, mantissa_bits: int) -> int:
    """Largest T with m + q*T <= mantissa_bits."""
    return (mantissa_bits - m) // q


# ----------------------------------------------------------------------------
# Workload mixes for the batched and the serving configurations.
# ----------------------------------------------------------------------------

def batch_mix(seed: int, n_grids: int = 64, side_lo: int = 256, side_hi: int = 4096,
              steps: int = 200):
    """Specs of independent 2D star grids: sides U{lo..hi} per axis, r in {1, 2}.

    Returns a list of dicts with keys ndim, radius, box, interior, steps, seed.
    """
    rng = np.random.default_rng(seed)
    out = []
    for j in range(n_grids):
        s0, s1 = (int(v) for v in rng.integers(side_lo, side_hi + 1, size=2))
        r = int(rng.integers(1, 3))
        out.append(dict(ndim=2, radius=r, box=False, interior=(s0, s1), steps=steps,
                        seed=item_seed(seed, j)))
    return out


def serve_mix(seed: int, n_requests: int, rate_per_s: float,
              side2d=(512, 8192), side3d=(64, 256), steps=(10, 1000)):
    """Poisson stream of mixed stencil requests.

    50% 2D (sides U{side2d} per axis) and 50% 3D (sides U{side3d}); star/box
    50/50; radius in {1, 2}; steps U{steps}; float32/float64 50/50.
    Arrival times are cumulative exponential gaps with mean 1/rate.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for j in range(n_requests):
        t += float(rng.exponential(1.0 / rate_per_s))
        ndim = 2 if rng.random() < 0.5 else 3
        lo, hi = side2d if ndim == 2 else side3d
        interior = tuple(int(v) for v in rng.integers(lo, hi + 1, size=ndim))
        out.append(dict(arrival=t, ndim=ndim, radius=int(rng.integers(1, 3)),
                        box=bool(rng.random() < 0.5), interior=interior,
                        steps=int(rng.integers(steps[0], steps[1] + 1)),
                        dtype="f32" if rng.random() < 0.5 else "f64",
                        seed=item_seed(seed, j)))
    return out
