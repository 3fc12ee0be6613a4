"""ctypes binding of libstencil5d.so (argument marshalling only).

Every step of the sweep runs in the library's HIP kernels; this module only
converts Python values into the C structs of ``include/stencil5d.h`` and
passes raw device pointers and a stream handle through.  PyTorch supplies the
device memory and the streams.  There is no fallback: if the library is not
built, or no GPU is present, calls fail with an exception.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libstencil5d.so")

S5D_OK, S5D_EINVAL, S5D_EUNSUPPORTED, S5D_ENOMEM, S5D_EDEVICE, S5D_EBUDGET, S5D_ECANCELED, S5D_ETIMEDOUT = range(8)
STAR, BOX = 0, 1
F32, F64 = 0, 1
ACC_PLAIN, ACC_COMPENSATED = 0, 1
EXPR_LINEAR, EXPR_DIV, EXPR_GRADIENT, EXPR_VARCOEF = range(4)

# Every symbol include/stencil5d.h declares.
EXPORTS = ("s5d_plan_create", "s5d_plan_destroy", "s5d_plan_query", "s5d_run", "s5d_run_fields",
           "s5d_batch_create", "s5d_batch_run", "s5d_batch_query", "s5d_batch_status",
           "s5d_batch_set_wait_limit", "s5d_batch_persistent_info", "s5d_batch_destroy",
           "s5d_run_batch",
           "s5d_server_create", "s5d_server_destroy", "s5d_server_now", "s5d_server_submit",
           "s5d_server_tick", "s5d_server_cancel", "s5d_server_sync", "s5d_server_request", "s5d_server_fetch",
           "s5d_server_get_stats",
           "s5d_plan_model", "s5d_autotune", "s5d_tune_cache_save", "s5d_tune_cache_load",
           "s5d_tune_cache_clear",
           "s5d_error_norms_workspace_bytes", "s5d_error_norms", "s5d_error_norms_noalloc",
           "s5d_status_string", "s5d_last_error")
NORMS_COUNT = 5
BATCH_GRAPH = 1
BATCH_PERSISTENT = 2


class S5DDesc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("ndim", ctypes.c_int32),
                ("radius", ctypes.c_int32), ("shape", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("accum", ctypes.c_int32),
                ("interior", ctypes.c_int64 * 3), ("steps", ctypes.c_int64),
                ("coeffs", ctypes.POINTER(ctypes.c_double)), ("n_coeffs", ctypes.c_int64),
                ("expr", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class S5DTuning(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("bt", ctypes.c_int32),
                ("tile0", ctypes.c_int32), ("tile1", ctypes.c_int32),
                ("stream_chunk", ctypes.c_int32), ("cells_per_lane", ctypes.c_int32),
                ("rows_per_wave", ctypes.c_int32), ("waves_per_eu", ctypes.c_int32),
                ("kernel", ctypes.c_int32)]


class S5DServerConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_running", ctypes.c_int32),
                ("hbm_budget_bytes", ctypes.c_int64), ("rounds_per_tick", ctypes.c_int32),
                ("n_streams", ctypes.c_int32), ("fail_admit_every", ctypes.c_int32),
                ("fail_tick_every", ctypes.c_int32)]


class S5DRequestInfo(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("state", ctypes.c_int32),
                ("result_index", ctypes.c_int32), ("status", ctypes.c_int32),
                ("updates", ctypes.c_int64), ("rounds_done", ctypes.c_int64),
                ("t_arrival", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("init_in_use", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class S5DServerStats(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("reserved", ctypes.c_int32),
                ("submitted", ctypes.c_int64), ("queued", ctypes.c_int64),
                ("running", ctypes.c_int64), ("done", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("bytes_in_use", ctypes.c_int64), ("bytes_peak", ctypes.c_int64),
                ("ticks", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("updates_done", ctypes.c_int64), ("latency_p50", ctypes.c_double),
                ("latency_p99", ctypes.c_double), ("makespan", ctypes.c_double)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_RELEASED, REQ_FAILED = range(5)


class S5DModel(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("bound", ctypes.c_int32),
                ("seconds", ctypes.c_double), ("t_alu", ctypes.c_double),
                ("t_hbm", ctypes.c_double), ("t_lds", ctypes.c_double),
                ("eff_cu", ctypes.c_double), ("hbm_bytes", ctypes.c_double),
                ("valu_ops", ctypes.c_double), ("workgroups", ctypes.c_int64)]


class S5DTuneReport(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n_candidates", ctypes.c_int32),
                ("n_measured", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("model_best_seconds", ctypes.c_double),
                ("best_seconds_per_step", ctypes.c_double),
                ("default_seconds_per_step", ctypes.c_double)]


class Stencil5DError(RuntimeError):
    def __init__(self, status, where, detail):
        self.status = status
        super().__init__("%s: %s (%s)" % (where, status_string(status), detail))


_lock = threading.Lock()
_lib = None


def load():
    """Load libstencil5d.so (once); raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libstencil5d.so is not built (%s); run "
                               "`python -m paper_2001_01473_amd.build`" % LIB_PATH)
        # One HIP runtime per process: PyTorch ships its own libamdhip64.so.7
        # and the library binds to whichever copy is loaded first, so torch
        # (which provides the device memory and streams) is loaded before it.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        lib.s5d_plan_create.restype = ctypes.c_int32
        lib.s5d_plan_create.argtypes = [ctypes.POINTER(S5DDesc), ctypes.POINTER(S5DTuning),
                                        ctypes.POINTER(vp)]
        lib.s5d_plan_destroy.restype = None
        lib.s5d_plan_destroy.argtypes = [vp]
        lib.s5d_plan_query.restype = ctypes.c_int32
        lib.s5d_plan_query.argtypes = [vp, ctypes.POINTER(S5DTuning),
                                       ctypes.POINTER(ctypes.c_int64)]
        lib.s5d_run.restype = ctypes.c_int32
        lib.s5d_run.argtypes = [vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int32)]
        lib.s5d_run_fields.restype = ctypes.c_int32
        lib.s5d_run_fields.argtypes = [vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_int32)]
        vpp = ctypes.POINTER(vp)
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.s5d_batch_create.restype = ctypes.c_int32
        lib.s5d_batch_create.argtypes = [vpp, vpp, vpp, ctypes.c_int32, ctypes.c_int32, vpp]
        lib.s5d_batch_run.restype = ctypes.c_int32
        lib.s5d_batch_run.argtypes = [vp, vp, i32p]
        lib.s5d_batch_query.restype = ctypes.c_int32
        lib.s5d_batch_query.argtypes = [vp, i32p, i32p]
        lib.s5d_batch_status.restype = ctypes.c_int32
        lib.s5d_batch_status.argtypes = [vp, vp]
        lib.s5d_batch_set_wait_limit.restype = ctypes.c_int32
        lib.s5d_batch_set_wait_limit.argtypes = [vp, ctypes.c_int64]
        lib.s5d_batch_persistent_info.restype = ctypes.c_int32
        lib.s5d_batch_persistent_info.argtypes = [vp, i32p, ctypes.POINTER(ctypes.c_int64),
                                                  ctypes.POINTER(ctypes.c_int64)]
        lib.s5d_batch_destroy.restype = None
        lib.s5d_batch_destroy.argtypes = [vp]
        lib.s5d_run_batch.restype = ctypes.c_int32
        lib.s5d_run_batch.argtypes = [vpp, vpp, vpp, ctypes.c_int32, vp, i32p]
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        lib.s5d_server_create.restype = ctypes.c_int32
        lib.s5d_server_create.argtypes = [ctypes.POINTER(S5DServerConfig), vpp]
        lib.s5d_server_destroy.restype = None
        lib.s5d_server_destroy.argtypes = [vp]
        lib.s5d_server_now.restype = ctypes.c_int32
        lib.s5d_server_now.argtypes = [vp, dp]
        lib.s5d_server_submit.restype = ctypes.c_int32
        lib.s5d_server_submit.argtypes = [vp, vp, vp, ctypes.c_double, ctypes.c_int32, i64p]
        lib.s5d_server_tick.restype = ctypes.c_int32
        lib.s5d_server_tick.argtypes = [vp, i32p, i32p]
        lib.s5d_server_cancel.restype = ctypes.c_int32
        lib.s5d_server_cancel.argtypes = [vp, ctypes.c_int64]
        lib.s5d_server_sync.restype = ctypes.c_int32
        lib.s5d_server_sync.argtypes = [vp]
        lib.s5d_server_request.restype = ctypes.c_int32
        lib.s5d_server_request.argtypes = [vp, ctypes.c_int64, ctypes.POINTER(S5DRequestInfo)]
        lib.s5d_server_fetch.restype = ctypes.c_int32
        lib.s5d_server_fetch.argtypes = [vp, ctypes.c_int64, vp]
        lib.s5d_server_get_stats.restype = ctypes.c_int32
        lib.s5d_server_get_stats.argtypes = [vp, ctypes.POINTER(S5DServerStats)]
        lib.s5d_plan_model.restype = ctypes.c_int32
        lib.s5d_plan_model.argtypes = [vp, ctypes.POINTER(S5DModel)]
        lib.s5d_autotune.restype = ctypes.c_int32
        lib.s5d_autotune.argtypes = [ctypes.POINTER(S5DDesc), ctypes.c_int32, vp,
                                     ctypes.POINTER(S5DTuning), ctypes.POINTER(S5DTuneReport)]
        lib.s5d_tune_cache_save.restype = ctypes.c_int32
        lib.s5d_tune_cache_save.argtypes = [ctypes.c_char_p]
        lib.s5d_tune_cache_load.restype = ctypes.c_int32
        lib.s5d_tune_cache_load.argtypes = [ctypes.c_char_p]
        lib.s5d_tune_cache_clear.restype = None
        lib.s5d_tune_cache_clear.argtypes = []
        lib.s5d_error_norms_workspace_bytes.restype = ctypes.c_int64
        lib.s5d_error_norms_workspace_bytes.argtypes = [ctypes.c_int64]
        lib.s5d_error_norms.restype = ctypes.c_int32
        lib.s5d_error_norms.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_int64,
                                        vp, vp, ctypes.c_int64, vp]
        lib.s5d_error_norms_noalloc.restype = ctypes.c_int32
        lib.s5d_error_norms_noalloc.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_int64,
                                                vp, vp]
        lib.s5d_status_string.restype = ctypes.c_char_p
        lib.s5d_status_string.argtypes = [ctypes.c_int32]
        lib.s5d_last_error.restype = ctypes.c_char_p
        lib.s5d_last_error.argtypes = []
        _lib = lib
        return lib


def status_string(status: int) -> str:
    return load().s5d_status_string(int(status)).decode()


def last_error() -> str:
    return load().s5d_last_error().decode()


def check(status: int, where: str):
    if status != S5D_OK:
        raise Stencil5DError(status, where, last_error())


def make_desc(ndim, radius, box, dtype, accum, interior, steps, coeffs, expr=EXPR_LINEAR):
    c = np.ascontiguousarray(np.asarray([] if coeffs is None else coeffs, dtype=np.float64).ravel())
    d = S5DDesc()
    d.struct_size = ctypes.sizeof(S5DDesc)
    d.ndim = int(ndim)
    d.radius = int(radius)
    d.shape = BOX if box else STAR
    d.dtype = int(dtype)
    d.accum = int(accum)
    ext = list(interior) + [1] * (3 - len(interior))
    for a in range(3):
        d.interior[a] = int(ext[a])
    d.steps = int(steps)
    d.coeffs = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if c.size else None
    d.n_coeffs = int(c.size)
    d.expr = int(expr)
    d.reserved = 0
    return d, c  # keep c alive while d is used


KERNELS = {"auto": 0, "blocked": 1, "direct": 2}


def make_tuning(bt=0, tile0=0, tile1=0, stream_chunk=0, cells_per_lane=0, rows_per_wave=0,
                waves_per_eu=0, kernel=0):
    t = S5DTuning()
    t.struct_size = ctypes.sizeof(S5DTuning)
    t.bt, t.tile0, t.tile1 = int(bt), int(tile0), int(tile1)
    t.stream_chunk, t.cells_per_lane = int(stream_chunk), int(cells_per_lane)
    t.rows_per_wave, t.waves_per_eu = int(rows_per_wave), int(waves_per_eu)
    t.kernel = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    return t
