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
from ._lib import (ACC_COMPENSATED, ACC_PLAIN, BOX, EXPR_DIV, EXPR_GRADIENT, EXPR_LINEAR,
                   EXPR_VARCOEF, F32, F64, STAR, Stencil5DError, last_error, status_string)

__all__ = ["Plan", "Batch", "Server", "solve", "error_norms", "error_norms_noalloc", "autotune", "tune_cache_save",
           "tune_cache_load", "tune_cache_clear", "NORM_NAMES", "Stencil5DError", "status_string",
           "last_error",
           "STAR", "BOX", "F32", "F64", "ACC_PLAIN", "ACC_COMPENSATED",
           "EXPR_LINEAR", "EXPR_DIV", "EXPR_GRADIENT", "EXPR_VARCOEF"]

_TUNING_KEYS = ("bt", "tile0", "tile1", "stream_chunk", "cells_per_lane", "rows_per_wave",
                "waves_per_eu", "kernel")


def _dtype_code(dtype):
    if isinstance(dtype, int) and dtype in (F32, F64):
        return dtype
    if dtype in ("f32", "float32"):
        return F32
    if dtype in ("f64", "float64"):
        return F64
    name = str(getattr(dtype, "__name__", dtype))
    if name.endswith("float32"):
        return F32
    if name.endswith("float64"):
        return F64
    raise ValueError("dtype must be float32 or float64, got %r" % (dtype,))


_EXPRS = {"linear": EXPR_LINEAR, "div": EXPR_DIV, "gradient": EXPR_GRADIENT, "varcoef": EXPR_VARCOEF}


def _expr_code(expr):
    if isinstance(expr, int) and expr in _EXPRS.values():
        return expr
    if expr in _EXPRS:
        return _EXPRS[expr]
    raise ValueError("expr must be one of %s" % sorted(_EXPRS))


def _accum_code(accum):
    if accum in (ACC_PLAIN, "plain"):
        return ACC_PLAIN
    if accum in (ACC_COMPENSATED, "compensated", "kahan"):
        return ACC_COMPENSATED
    raise ValueError("accum must be 'plain' or 'compensated'")


class Plan:
    """An immutable sweep plan (``s5d_plan``): stencil, extents, steps, blocking.

    ``expr`` selects what a step computes (``S5D_EXPR_*`` of the C header):
    "linear" (``coeffs``: the n weights), "div" (the n weights, then the
    divisor c0), "gradient" (cc, c0) or "varcoef" (no ``coeffs``; the
    per-cell weights are passed to ``run(..., fields=)``)."""

    def __init__(self, *, ndim, radius, box, dtype, interior, steps, coeffs=None,
                 accum="plain", expr="linear", **tuning):
        unknown = set(tuning) - set(_TUNING_KEYS)
        if unknown:
            raise TypeError("unknown tuning keys: %s" % sorted(unknown))
        lib = _lib.load()
        self.ndim, self.radius, self.box = int(ndim), int(radius), bool(box)
        self.dtype = _dtype_code(dtype)
        self.interior = tuple(int(i) for i in interior)
        self.steps = int(steps)
        self.expr = _expr_code(expr)
        desc, keep = _lib.make_desc(ndim, radius, box, self.dtype, _accum_code(accum),
                                    self.interior, steps, coeffs, self.expr)
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

    def model(self) -> dict:
        """The performance model's prediction for this plan's whole sweep."""
        m = _lib.S5DModel()
        m.struct_size = ctypes.sizeof(m)
        _lib.check(_lib.load().s5d_plan_model(self._h, ctypes.byref(m)), "s5d_plan_model")
        out = {k: getattr(m, k) for k, _ in m._fields_ if k != "struct_size"}
        out["bound"] = ("alu", "hbm", "lds")[m.bound]
        return out

    def run(self, buf0, buf1, stream=None, fields=None) -> int:
        """Enqueue the sweep; returns the index (0/1) of the buffer holding the
        result.  ``fields`` (variable-coefficient plans only): a contiguous
        device tensor of the plan's dtype and shape (n_points,) + interior."""
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
        if fields is None:
            _lib.check(_lib.load().s5d_run(self._h, ctypes.c_void_p(buf0.data_ptr()),
                                           ctypes.c_void_p(buf1.data_ptr()),
                                           ctypes.c_void_p(handle), ctypes.byref(idx)), "s5d_run")
            return int(idx.value)
        if not fields.is_cuda or not fields.is_contiguous() or _dtype_code(fields.dtype) != self.dtype:
            raise ValueError("fields must be a contiguous device tensor of the plan's dtype")
        if tuple(fields.shape[1:]) != self.interior:
            raise ValueError("fields must have shape (n_points,) + interior")
        _lib.check(_lib.load().s5d_run_fields(self._h, ctypes.c_void_p(buf0.data_ptr()),
                                              ctypes.c_void_p(buf1.data_ptr()),
                                              ctypes.c_void_p(fields.data_ptr()),
                                              ctypes.c_void_p(handle), ctypes.byref(idx)),
                   "s5d_run_fields")
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


def _stream_handle(stream, device):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _check_pair(plan, b0, b1):
    for b in (b0, b1):
        if not b.is_cuda or not b.is_contiguous():
            raise ValueError("buffers must be contiguous device tensors")
        if tuple(b.shape) != plan.padded_shape:
            raise ValueError("buffer shape %s != padded shape %s" % (tuple(b.shape), plan.padded_shape))
        if _dtype_code(b.dtype) != plan.dtype:
            raise ValueError("buffer dtype does not match the plan")


class Batch:
    """Many independent sweeps run together (``s5d_batch``): per round index,
    one launch per kernel variant over all grids, or (``persistent=True``) one
    persistent launch per stencil family over every round of its grids;
    optionally replayed as one HIP graph.  ``plans``, ``bufs0`` and ``bufs1``
    are equal-length lists; the buffers are bound to the batch and must outlive
    it."""

    def __init__(self, plans, bufs0, bufs1, *, graph=False, persistent=False):
        lib = _lib.load()
        n = len(plans)
        if not (len(bufs0) == len(bufs1) == n):
            raise ValueError("plans, bufs0 and bufs1 differ in length")
        for p, b0, b1 in zip(plans, bufs0, bufs1):
            _check_pair(p, b0, b1)
        vp = ctypes.c_void_p
        self.n = n
        self._device = bufs0[0].device if n else None
        self._bufs = (list(bufs0), list(bufs1))  # keep the tensors alive
        self._plans = list(plans)
        arr = vp * max(n, 1)
        hp = arr(*[p._h for p in plans])
        b0 = arr(*[vp(b.data_ptr()) for b in bufs0])
        b1 = arr(*[vp(b.data_ptr()) for b in bufs1])
        h = vp()
        flags = (_lib.BATCH_GRAPH if graph else 0) | (_lib.BATCH_PERSISTENT if persistent else 0)
        _lib.check(lib.s5d_batch_create(hp, b0, b1, n, flags, ctypes.byref(h)), "s5d_batch_create")
        self._h = h

    def run(self, stream=None):
        """Enqueue every grid's sweep; returns the list of result buffer indices."""
        if self._h is None:
            raise RuntimeError("batch destroyed")
        idx = (ctypes.c_int32 * max(self.n, 1))()
        handle = _stream_handle(stream, self._device) if self.n else 0
        _lib.check(_lib.load().s5d_batch_run(self._h, ctypes.c_void_p(handle), idx), "s5d_batch_run")
        return [int(idx[i]) for i in range(self.n)]

    def query(self) -> dict:
        lib = _lib.load()
        nl, ns = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(lib.s5d_batch_query(self._h, ctypes.byref(nl), ctypes.byref(ns)), "s5d_batch_query")
        pl, wg, it = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _lib.check(lib.s5d_batch_persistent_info(self._h, ctypes.byref(pl), ctypes.byref(wg), ctypes.byref(it)),
                   "s5d_batch_persistent_info")
        out = {"launches": int(nl.value), "round_steps": int(ns.value)}
        if pl.value:
            out.update(persistent_launches=int(pl.value), persistent_workgroups=int(wg.value),
                       persistent_items=int(it.value))
        return out

    def status(self, stream=None):
        """Synchronise the stream of the last run and raise Stencil5DError
        (S5D_ETIMEDOUT) if a persistent launch's bounded wait ran out."""
        handle = _stream_handle(stream, self._device) if self.n else 0
        _lib.check(_lib.load().s5d_batch_status(self._h, ctypes.c_void_p(handle)), "s5d_batch_status")

    def set_wait_limit(self, polls):
        """Most polls a persistent workgroup waits for its grid's previous round."""
        _lib.check(_lib.load().s5d_batch_set_wait_limit(self._h, int(polls)), "s5d_batch_set_wait_limit")

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.load().s5d_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune(*, ndim, radius, box, dtype, interior, steps, coeffs=None, accum="plain", top_k=4,
             stream=None, expr="linear"):
    """Model-ranked, GPU-measured choice of the blocking for this problem
    (``s5d_autotune``); returns (tuning dict, report dict).  The choice is
    cached for later plans of the same stencil and extent bucket."""
    lib = _lib.load()
    desc, keep = _lib.make_desc(ndim, radius, box, _dtype_code(dtype), _accum_code(accum),
                                interior, steps, coeffs, _expr_code(expr))
    best = _lib.make_tuning()
    rep = _lib.S5DTuneReport()
    rep.struct_size = ctypes.sizeof(rep)
    handle = _stream_handle(stream, None) if stream is not None else 0
    st = lib.s5d_autotune(ctypes.byref(desc), int(top_k), ctypes.c_void_p(handle),
                          ctypes.byref(best), ctypes.byref(rep))
    del keep
    _lib.check(st, "s5d_autotune")
    tun = {k: int(getattr(best, k)) for k in _TUNING_KEYS}
    report = {k: getattr(rep, k) for k, _ in rep._fields_ if k not in ("struct_size", "reserved")}
    return tun, report


def tune_cache_save(path):
    _lib.check(_lib.load().s5d_tune_cache_save(str(path).encode()), "s5d_tune_cache_save")


def tune_cache_load(path):
    _lib.check(_lib.load().s5d_tune_cache_load(str(path).encode()), "s5d_tune_cache_load")


def tune_cache_clear():
    _lib.load().s5d_tune_cache_clear()


class Server:
    """Serving loop with continuous batching (``s5d_server``): requests queue,
    are admitted under an HBM budget and advance one round per ``tick()``,
    all running requests together.  Times are seconds on the server clock."""

    def __init__(self, *, hbm_budget_bytes, max_running=0, rounds_per_tick=0, n_streams=0,
                 fail_admit_every=0, fail_tick_every=0):
        lib = _lib.load()
        cfg = _lib.S5DServerConfig()
        cfg.struct_size = ctypes.sizeof(cfg)
        cfg.max_running = int(max_running)
        cfg.hbm_budget_bytes = int(hbm_budget_bytes)
        cfg.rounds_per_tick = int(rounds_per_tick)
        cfg.n_streams = int(n_streams)
        cfg.fail_admit_every = int(fail_admit_every)
        cfg.fail_tick_every = int(fail_tick_every)
        h = ctypes.c_void_p()
        _lib.check(lib.s5d_server_create(ctypes.byref(cfg), ctypes.byref(h)), "s5d_server_create")
        self._h = h
        self._inits = {}  # request id -> initial grid, kept alive until the server has read it

    def now(self) -> float:
        t = ctypes.c_double()
        _lib.check(_lib.load().s5d_server_now(self._h, ctypes.byref(t)), "s5d_server_now")
        return float(t.value)

    def submit(self, plan, init, *, arrival=-1.0, keep_result=False) -> int:
        """Queue ``plan`` with initial grid ``init`` (a contiguous host numpy
        array or device tensor of the plan's padded shape); returns its id."""
        import numpy as np
        if hasattr(init, "data_ptr"):
            if not init.is_contiguous() or tuple(init.shape) != plan.padded_shape:
                raise ValueError("init must be a contiguous tensor of the padded shape")
            if _dtype_code(init.dtype) != plan.dtype:
                raise ValueError("init dtype does not match the plan")
            ptr = init.data_ptr()
        else:
            init = np.ascontiguousarray(init)
            if init.shape != plan.padded_shape or _dtype_code(init.dtype) != plan.dtype:
                raise ValueError("init must match the plan's padded shape and dtype")
            ptr = init.ctypes.data
        rid = ctypes.c_int64()
        _lib.check(_lib.load().s5d_server_submit(self._h, plan._h, ctypes.c_void_p(ptr),
                                                 float(arrival), int(bool(keep_result)),
                                                 ctypes.byref(rid)), "s5d_server_submit")
        self._inits[int(rid.value)] = init
        return int(rid.value)

    def tick(self):
        """Admit what fits, advance every running request by one round;
        returns (running, queued)."""
        nr, nq = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib.load().s5d_server_tick(self._h, ctypes.byref(nr), ctypes.byref(nq)),
                   "s5d_server_tick")
        self._drop_admitted()
        return int(nr.value), int(nq.value)

    def cancel(self, rid):
        """Cancel a queued or running request (it becomes FAILED with
        S5D_ECANCELED; a running one leaves at the next tick)."""
        _lib.check(_lib.load().s5d_server_cancel(self._h, int(rid)), "s5d_server_cancel")

    def sync(self):
        _lib.check(_lib.load().s5d_server_sync(self._h), "s5d_server_sync")
        self._drop_admitted()

    def request(self, rid) -> dict:
        info = _lib.S5DRequestInfo()
        info.struct_size = ctypes.sizeof(info)
        _lib.check(_lib.load().s5d_server_request(self._h, int(rid), ctypes.byref(info)),
                   "s5d_server_request")
        return {k: getattr(info, k) for k, _ in info._fields_ if k not in ("struct_size", "reserved")}

    def fetch(self, rid, out):
        """Copy a finished kept result into ``out`` (tensor or numpy array)."""
        ptr = out.data_ptr() if hasattr(out, "data_ptr") else out.ctypes.data
        _lib.check(_lib.load().s5d_server_fetch(self._h, int(rid), ctypes.c_void_p(ptr)),
                   "s5d_server_fetch")
        return out

    def stats(self) -> dict:
        st = _lib.S5DServerStats()
        st.struct_size = ctypes.sizeof(st)
        _lib.check(_lib.load().s5d_server_get_stats(self._h, ctypes.byref(st)),
                   "s5d_server_get_stats")
        return {k: getattr(st, k) for k, _ in st._fields_ if k not in ("struct_size", "reserved")}

    def _drop_admitted(self):
        # an initial grid may go once the server's copy of it has run
        for rid in sorted(self._inits):
            if not self.request(rid)["init_in_use"]:
                del self._inits[rid]

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.load().s5d_server_destroy(self._h)
            self._h = None
            self._inits.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(grid, *, radius, box, coeffs=None, steps, accum="plain", stream=None, expr="linear",
          fields=None, **tuning):
    """Run ``steps`` time steps on a padded device grid; returns the result tensor.

    ``grid`` (float32/float64, contiguous, on the GPU, boundary included) is
    used as buffer 0 and may be overwritten; the returned tensor is either
    ``grid`` itself or a second buffer allocated here.
    """
    import torch
    interior = tuple(s - 2 * radius for s in grid.shape)
    plan = Plan(ndim=grid.dim(), radius=radius, box=box, dtype=grid.dtype, interior=interior,
                steps=steps, coeffs=coeffs, accum=accum, expr=expr, **tuning)
    other = torch.empty_like(grid)
    idx = plan.run(grid, other, stream=stream, fields=fields)
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


def error_norms_noalloc(got, ref, out, *, stream=None):
    """``error_norms`` through ``s5d_error_norms_noalloc``: the partials go to
    the library's fixed per-device scratch, so neither this call nor the
    library allocates.  ``out`` (a float64 device tensor of NORMS_COUNT
    values on the current device) receives the result and is returned.  Calls
    that overlap on one GPU race on that scratch."""
    import torch
    lib = _lib.load()
    for t in (got, ref, out):
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError("got, ref and out must be contiguous device tensors")
    n = got.numel()
    if ref.numel() != n:
        raise ValueError("got and ref differ in size")
    if out.dtype != torch.float64 or out.numel() < _lib.NORMS_COUNT:
        raise ValueError("out must be a float64 tensor of %d values" % _lib.NORMS_COUNT)
    if stream is None:
        stream = torch.cuda.current_stream(got.device)
    handle = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    _lib.check(lib.s5d_error_norms_noalloc(ctypes.c_void_p(got.data_ptr()), _dtype_code(got.dtype),
                                           ctypes.c_void_p(ref.data_ptr()), _dtype_code(ref.dtype),
                                           int(n), ctypes.c_void_p(out.data_ptr()),
                                           ctypes.c_void_p(handle)), "s5d_error_norms_noalloc")
    return out
