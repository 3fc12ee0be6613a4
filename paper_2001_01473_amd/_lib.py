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

S5D_OK, S5D_EINVAL, S5D_EUNSUPPORTED, S5D_ENOMEM, S5D_EDEVICE, S5D_EBUDGET = range(6)
STAR, BOX = 0, 1
F32, F64 = 0, 1
ACC_PLAIN, ACC_COMPENSATED = 0, 1

# Every symbol include/stencil5d.h declares.
EXPORTS = ("s5d_plan_create", "s5d_plan_destroy", "s5d_plan_query", "s5d_run",
           "s5d_error_norms_workspace_bytes", "s5d_error_norms",
           "s5d_status_string", "s5d_last_error")
NORMS_COUNT = 5


class S5DDesc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("ndim", ctypes.c_int32),
                ("radius", ctypes.c_int32), ("shape", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("accum", ctypes.c_int32),
                ("interior", ctypes.c_int64 * 3), ("steps", ctypes.c_int64),
                ("coeffs", ctypes.POINTER(ctypes.c_double)), ("n_coeffs", ctypes.c_int64)]


class S5DTuning(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("bt", ctypes.c_int32),
                ("tile0", ctypes.c_int32), ("tile1", ctypes.c_int32),
                ("stream_chunk", ctypes.c_int32), ("cells_per_lane", ctypes.c_int32),
                ("rows_per_wave", ctypes.c_int32), ("waves_per_eu", ctypes.c_int32)]


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
        lib.s5d_error_norms_workspace_bytes.restype = ctypes.c_int64
        lib.s5d_error_norms_workspace_bytes.argtypes = [ctypes.c_int64]
        lib.s5d_error_norms.restype = ctypes.c_int32
        lib.s5d_error_norms.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_int64,
                                        vp, vp, ctypes.c_int64, vp]
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


def make_desc(ndim, radius, box, dtype, accum, interior, steps, coeffs):
    c = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
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
    d.coeffs = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.n_coeffs = int(c.size)
    return d, c  # keep c alive while d is used


def make_tuning(bt=0, tile0=0, tile1=0, stream_chunk=0, cells_per_lane=0, rows_per_wave=0,
                waves_per_eu=0):
    t = S5DTuning()
    t.struct_size = ctypes.sizeof(S5DTuning)
    t.bt, t.tile0, t.tile1 = int(bt), int(tile0), int(tile1)
    t.stream_chunk, t.cells_per_lane = int(stream_chunk), int(cells_per_lane)
    t.rows_per_wave, t.waves_per_eu = int(rows_per_wave), int(waves_per_eu)
    return t
