"""CPU oracle for the stencil sweep -- test infrastructure only.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
this package; the GPU library never imports, links or calls it, and it
imports nothing from the GPU library.

The arithmetic lives in ``oracle.c`` (plain C, no fused multiply-add, OpenMP
over axis 0): the naive double-buffered time loop of AN5D's input programs
(Fig. 4; "Host Code" under "Code Generation") applied to the synthetic
star/box stencils of Table 3.  This module only loads that library, builds it
with gcc when it is missing, and marshals numpy arrays.

Every function here is pinned by ``tests/test_oracle_pins.py`` against exact
dyadic arithmetic, exact rational brute force, closed-form eigenmodes,
scipy's correlate/convolve and structural invariants; the compensated float32
variant against exact rational sums and the published error bound of the
compensated dot product.  The expression stencils of the paper's general
benchmarks (Table 3: a weighted sum divided by a constant, and gradient2d)
and the variable-coefficient sweep are pinned in ``tests/test_oracle_expr.py``
(the Fig. 4 program's impulse response, exact dyadic arithmetic, closed-form
fields, a high-precision decimal brute force and exact rational matrix
powers).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

# gcc flags: no contraction into FMA and no fast-math, so the term order in
# oracle.c is the order the hardware executes.
CFLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-std=c11"]


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` next to it; returns its path."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH):
                build(force=False)
            lib = ctypes.CDLL(_LIB_PATH)
            i64p = ctypes.POINTER(ctypes.c_int64)
            lib.oracle_offsets.restype = ctypes.c_int
            lib.oracle_offsets.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_void_p]
            for name in ("oracle_sweep_f64", "oracle_sweep_f32", "oracle_sweep_f32_dot2"):
                fn = getattr(lib, name)
                fn.restype = ctypes.c_int
                fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, i64p,
                               ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
            for name, real in (("oracle_sweep_div_f64", ctypes.c_double),
                               ("oracle_sweep_div_f32", ctypes.c_float)):
                fn = getattr(lib, name)
                fn.restype = ctypes.c_int
                fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, i64p,
                               ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, real,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
            for name, real in (("oracle_sweep_gradient_f64", ctypes.c_double),
                               ("oracle_sweep_gradient_f32", ctypes.c_float)):
                fn = getattr(lib, name)
                fn.restype = ctypes.c_int
                fn.argtypes = [i64p, ctypes.c_int64, real, real, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_int]
            for name in ("oracle_sweep_varcoef_f64", "oracle_sweep_varcoef_f32"):
                fn = getattr(lib, name)
                fn.restype = ctypes.c_int
                fn.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, i64p,
                               ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p, ctypes.c_int]
            lib.oracle_max_threads.restype = ctypes.c_int
            lib.oracle_max_threads.argtypes = []
            _lib = lib
    return _lib


def offsets(ndim: int, radius: int, box: bool) -> np.ndarray:
    """Canonical stencil offsets, shape (n, ndim): lexicographic in (d0, d1[, d2])."""
    lib = _load()
    n = lib.oracle_offsets(ndim, radius, int(bool(box)), None)
    if n < 0:
        raise ValueError("unsupported stencil ndim=%r radius=%r" % (ndim, radius))
    out = np.zeros((n, 3), dtype=np.int32)
    lib.oracle_offsets(ndim, radius, int(bool(box)), out.ctypes.data)
    return out[:, :ndim].copy()


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def sweep(a0: np.ndarray, *, radius: int, box: bool, coeffs, steps: int,
          threads: int = 0, accum: str = "plain") -> np.ndarray:
    """Run T = ``steps`` steps of the naive double-buffered loop.

    ``a0`` is the padded initial grid (boundary included), float64 or float32;
    the working precision is ``a0.dtype`` and ``coeffs`` are cast to it.
    ``accum="compensated"`` (float32 only) sums each cell's terms with the
    compensated dot product (Dot2) instead of plain left-to-right addition.
    Returns a new array holding A[T % 2] (the input is not modified).
    ``threads`` = 0 keeps OpenMP's default.
    """
    a0 = np.asarray(a0)
    if accum not in ("plain", "compensated"):
        raise ValueError("accum must be 'plain' or 'compensated'")
    if accum == "compensated":
        if a0.dtype != np.float32:
            raise TypeError("compensated accumulation is defined for float32 grids")
        fn, ct = _load().oracle_sweep_f32_dot2, np.float32
    elif a0.dtype == np.float64:
        fn, ct = _load().oracle_sweep_f64, np.float64
    elif a0.dtype == np.float32:
        fn, ct = _load().oracle_sweep_f32, np.float32
    else:
        raise TypeError("oracle works on float64 or float32 grids, got %s" % a0.dtype)
    ndim = a0.ndim
    if ndim not in (2, 3):
        raise ValueError("grid must be 2D or 3D")
    interior = np.array([s - 2 * radius for s in a0.shape] + [1] * (3 - ndim),
                        dtype=np.int64)
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64).astype(ct))
    b0 = np.ascontiguousarray(a0).copy()
    b1 = np.empty_like(b0)
    rc = fn(ndim, radius, int(bool(box)),
            interior.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            int(steps), c.ctypes.data, int(c.size), b0.ctypes.data, b1.ctypes.data,
            int(threads))
    if rc < 0:
        raise ValueError("oracle rejected the arguments (ndim=%d radius=%d n_coeffs=%d "
                         "steps=%d shape=%s)" % (ndim, radius, c.size, steps, a0.shape))
    return b0 if rc == 0 else b1


def _prep(a0, radius):
    a0 = np.asarray(a0)
    if a0.dtype not in (np.float64, np.float32):
        raise TypeError("oracle works on float64 or float32 grids, got %s" % a0.dtype)
    if a0.ndim not in (2, 3):
        raise ValueError("grid must be 2D or 3D")
    interior = np.array([s - 2 * radius for s in a0.shape] + [1] * (3 - a0.ndim), dtype=np.int64)
    b0 = np.ascontiguousarray(a0).copy()
    return a0.dtype, interior, b0, np.empty_like(b0)


def sweep_div(a0: np.ndarray, *, radius: int, box: bool, coeffs, divisor, steps: int,
              threads: int = 0) -> np.ndarray:
    """Expression stencil "weighted sum / c0" (Table 3: j2d5pt, j2d9pt,
    j2d9pt-gol, j3d27pt): each step every interior cell becomes the canonical
    left-to-right sum of c_k times its neighbour, divided by ``divisor``, in
    the grid's precision.  Returns A[T % 2]."""
    dt, interior, b0, b1 = _prep(a0, radius)
    real = np.float64 if dt == np.float64 else np.float32
    fn = _load().oracle_sweep_div_f64 if dt == np.float64 else _load().oracle_sweep_div_f32
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64).astype(real))
    rc = fn(a0.ndim, radius, int(bool(box)), interior.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            int(steps), c.ctypes.data, int(c.size), float(real(divisor)), b0.ctypes.data,
            b1.ctypes.data, int(threads))
    if rc < 0:
        raise ValueError("oracle rejected the arguments")
    return b0 if rc == 0 else b1


def sweep_gradient(a0: np.ndarray, *, cc, c0, steps: int, threads: int = 0) -> np.ndarray:
    """gradient2d (Table 3), radius 1: each step every interior cell becomes
    cc * f + 1 / sqrt(c0 + sum over its four axis neighbours n of (f - f_n)^2),
    the squares added to c0 in canonical offset order.  Returns A[T % 2]."""
    dt, interior, b0, b1 = _prep(a0, 1)
    if a0.ndim != 2:
        raise ValueError("gradient2d is a 2D stencil")
    real = np.float64 if dt == np.float64 else np.float32
    fn = _load().oracle_sweep_gradient_f64 if dt == np.float64 else _load().oracle_sweep_gradient_f32
    rc = fn(interior.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(steps), float(real(cc)),
            float(real(c0)), b0.ctypes.data, b1.ctypes.data, int(threads))
    if rc < 0:
        raise ValueError("oracle rejected the arguments")
    return b0 if rc == 0 else b1


def sweep_varcoef(a0: np.ndarray, *, radius: int, box: bool, cfield, steps: int,
                  threads: int = 0) -> np.ndarray:
    """Variable-coefficient sweep: every interior cell q has its own weights,
    A'[q] = sum_k cfield[k][q] * A[q + o_k] in canonical order.  ``cfield``
    has shape (n_points,) + interior extents and the grid's dtype.  Returns
    A[T % 2]."""
    dt, interior, b0, b1 = _prep(a0, radius)
    n = offsets(a0.ndim, radius, box).shape[0]
    cf = np.ascontiguousarray(np.asarray(cfield, dtype=dt))
    if cf.shape != (n,) + tuple(int(i) for i in interior[:a0.ndim]):
        raise ValueError("cfield must have shape (n_points,) + interior extents")
    fn = _load().oracle_sweep_varcoef_f64 if dt == np.float64 else _load().oracle_sweep_varcoef_f32
    rc = fn(a0.ndim, radius, int(bool(box)), interior.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            int(steps), cf.ctypes.data, b0.ctypes.data, b1.ctypes.data, int(threads))
    if rc < 0:
        raise ValueError("oracle rejected the arguments")
    return b0 if rc == 0 else b1
