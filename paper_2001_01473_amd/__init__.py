"""stencil5d: temporally blocked Jacobi-style stencil sweeps on MI355X (gfx950).

The compute path is libstencil5d.so (hand-written HIP kernels behind the C
ABI of ``include/stencil5d.h``); this package is its thin Python binding.
PyTorch provides device memory and streams.  Importing the package loads
nothing; the library is loaded on first use and its absence is an error.

    import torch, paper_2001_01473_amd as s5d
    out = s5d.solve(grid_cuda, radius=1, box=False, coeffs=c, steps=1000)
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (ACC_COMPENSATED, ACC_PLAIN, BOX, F32, F64, STAR, Stencil5DError,
                   last_error, status_string)

__all__ = ["Plan", "solve", "error_norms", "NORM_NAMES", "Stencil5DError", "status_string",
           "last_error",
           "STAR", "BOX", "F32", "F64", "ACC_PLAIN", "ACC_COMPENSATED"]

_TUNING_KEYS = ("bt", "tile0", "tile1", "stream_chunk", "cells_per_lane", "rows_per_wave",
                "waves_per_eu")


def _dtype_code(dtype):
    if dtype in (F32, "f32", "float32"):
        return F32
    if dtype in (F64, "f64", "float64"):
        return F64
    name = str(dtype)
    if name.endswith("float32"):
        return F32
    if name.endswith("float64"):
        return F64
    raise ValueError("dtype must be float32 or float64, got %r" % (dtype,))


def _accum_code(accum):
    if accum in (ACC_PLAIN, "plain"):
        return ACC_PLAIN
    if accum in (ACC_COMPENSATED, "compensated", "kahan"):
        return ACC_COMPENSATED
    raise ValueError("accum must be 'plain' or 'compensated'")


class Plan:
    """An immutable sweep plan (``s5d_plan``): stencil, extents, steps, blocking."""

    def __init__(self, *, ndim, radius, box, dtype, interior, steps, coeffs,
                 accum="plain", **tuning):
        unknown = set(tuning) - set(_TUNING_KEYS)
        if unknown:
            raise TypeError("unknown tuning keys: %s" % sorted(unknown))
        lib = _lib.load()
        self.ndim, self.radius, self.box = int(ndim), int(radius), bool(box)
        self.dtype = _dtype_code(dtype)
        self.interior = tuple(int(i) for i in interior)
        self.steps = int(steps)
        desc, keep = _lib.make_desc(ndim, radius, box, self.dtype, _accum_code(accum),
                                    self.interior, steps, coeffs)
        tun = _lib.make_tuning(**tuning) if tuning else None
        h = ctypes.c_void_p()
        st = lib.s5d_plan_create(ctypes.byref(desc), ctypes.byref(tun) if tun else None,
                                 ctypes.byref(h))
        del keep
        _lib.check(st, "s5d_plan_create")
        self._h = h

    @property
    def padded_shape(self):
        return tuple(i + 2 * self.radius for i in self.interior)

    def query(self) -> dict:
        t = _lib.make_tuning()
        nbytes = ctypes.c_int64()
        _lib.check(_lib.load().s5d_plan_query(self._h, ctypes.byref(t), ctypes.byref(nbytes)),
                   "s5d_plan_query")
        out = {k: int(getattr(t, k)) for k in _TUNING_KEYS}
        out["bytes_per_buffer"] = int(nbytes.value)
        return out

    def run(self, buf0, buf1, stream=None) -> int:
        """Enqueue the sweep; returns the index (0/1) of the buffer holding the result."""
        if self._h is None:
            raise RuntimeError("plan destroyed")
        import torch
        for b in (buf0, buf1):
            if not b.is_cuda or not b.is_contiguous():
                raise ValueError("buffers must be contiguous device tensors")
            if tuple(b.shape) != self.padded_shape:
                raise ValueError("buffer shape %s != padded shape %s"
                                 % (tuple(b.shape), self.padded_shape))
            if _dtype_code(b.dtype) != self.dtype:
                raise ValueError("buffer dtype does not match the plan")
        if stream is None:
            stream = torch.cuda.current_stream(buf0.device)
        handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        idx = ctypes.c_int32(-1)
        _lib.check(_lib.load().s5d_run(self._h, ctypes.c_void_p(buf0.data_ptr()),
                                       ctypes.c_void_p(buf1.data_ptr()),
                                       ctypes.c_void_p(handle), ctypes.byref(idx)), "s5d_run")
        return int(idx.value)

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.load().s5d_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(grid, *, radius, box, coeffs, steps, accum="plain", stream=None, **tuning):
    """Run ``steps`` time steps on a padded device grid; returns the result tensor.

    ``grid`` (float32/float64, contiguous, on the GPU, boundary included) is
    used as buffer 0 and may be overwritten; the returned tensor is either
    ``grid`` itself or a second buffer allocated here.
    """
    import torch
    interior = tuple(s - 2 * radius for s in grid.shape)
    plan = Plan(ndim=grid.dim(), radius=radius, box=box, dtype=grid.dtype, interior=interior,
                steps=steps, coeffs=coeffs, accum=accum, **tuning)
    other = torch.empty_like(grid)
    idx = plan.run(grid, other, stream=stream)
    plan.close()
    return grid if idx == 0 else other


# Order of the values s5d_error_norms writes.
NORM_NAMES = ("max_abs_err", "max_abs_ref", "max_rel_err", "rms_err", "rms_ref")


def error_norms(got, ref, *, stream=None, out=None, workspace=None):
    """Float64 error norms of device tensor ``got`` against device tensor
    ``ref`` (same number of elements, float32 or float64), computed on the GPU
    by ``s5d_error_norms``.  Returns a float64 device tensor of the five values
    in NORM_NAMES order (``out`` if given); ``workspace`` (a device tensor of at
    least ``s5d_error_norms_workspace_bytes`` bytes) is allocated if omitted."""
    import torch
    lib = _lib.load()
    for t in (got, ref):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("got and ref must be contiguous device tensors")
    n = got.numel()
    if ref.numel() != n:
        raise ValueError("got and ref differ in size")
    need = int(lib.s5d_error_norms_workspace_bytes(n))
    if out is None:
        out = torch.empty(_lib.NORMS_COUNT, dtype=torch.float64, device=got.device)
    if workspace is None:
        workspace = torch.empty(max(need, 8), dtype=torch.uint8, device=got.device)
    if stream is None:
        stream = torch.cuda.current_stream(got.device)
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    _lib.check(lib.s5d_error_norms(ctypes.c_void_p(got.data_ptr()), _dtype_code(got.dtype),
                                   ctypes.c_void_p(ref.data_ptr()), _dtype_code(ref.dtype),
                                   int(n), ctypes.c_void_p(out.data_ptr()),
                                   ctypes.c_void_p(workspace.data_ptr()),
                                   int(workspace.numel() * workspace.element_size()),
                                   ctypes.c_void_p(handle)), "s5d_error_norms")
    return out
