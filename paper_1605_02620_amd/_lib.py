"""ctypes declarations of librsos.so (include/rsos.h).

Loads the in-tree library built by paper_1605_02620_amd/build.py.  torch is
imported first so that the library binds to the same HIP runtime as torch
(both use the soname libamdhip64.so.7).  There is no fallback: without the
built library every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (HIP runtime shared with the library)

_PKG = os.path.dirname(os.path.abspath(__file__))
# RSOS_LIBRARY selects another build of the same library (e.g. to compare
# compile-time variants); by default the in-tree build is used.
SO_PATH = os.environ.get("RSOS_LIBRARY") or os.path.join(_PKG, "librsos.so")

c_i32, c_i64, c_u32, c_u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
c_vp = ctypes.c_void_p
P = ctypes.POINTER

OK, E_INVAL, E_RSOS, E_OVERFLOW, E_DEVICE, E_NOMEM, E_STATE, E_BUSY = 0, -1, -2, -3, -4, -5, -6, -7
JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_CANCELLED = 0, 1, 2, 3
FLAG_PACKED16 = 1
FLAG_DT4 = 2
FLAG_TUNE = 4
STATIC_MAX_SWEEPS = 4096


class Params(ctypes.Structure):
    _fields_ = [("L", c_i32), ("N", c_i32), ("D", c_i32), ("flags", c_i32), ("seed", c_u64)]


class Width(ctypes.Structure):
    _fields_ = [("t", c_i64), ("s1", c_i64), ("s2", c_i64), ("accepted", c_i64), ("w2", ctypes.c_double)]


class Moments(ctypes.Structure):
    _fields_ = [("t", c_i64), ("ref", c_i64), ("c1", c_i64), ("c2", c_i64), ("c3", c_u64 * 2),
                ("c4", c_u64 * 2), ("phi2", ctypes.c_double), ("phi3", ctypes.c_double),
                ("phi4", ctypes.c_double)]

    def as_dict(self):
        def i128(a):
            v = (int(a[1]) << 64) | int(a[0])
            return v - (1 << 128) if v >> 127 else v
        return {"t": self.t, "ref": self.ref, "c1": self.c1, "c2": self.c2, "c3": i128(self.c3),
                "c4": i128(self.c4), "phi2": self.phi2, "phi3": self.phi3, "phi4": self.phi4}


class Tune(ctypes.Structure):
    _fields_ = [("TX", c_i32), ("TY", c_i32), ("NT", c_i32), ("elem", c_i32), ("xmode", c_i32),
                ("graph_sweeps", c_i32), ("candidates", c_i32), ("measured", c_i32),
                ("ms_per_sweep", ctypes.c_double), ("ms_first_fit", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class RsosError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"rsos status {status}: {msg}")
        self.status = status


# (name, restype, argtypes) for every entry point of include/rsos.h
SIGNATURES = [
    ("rsos_init", c_i32, [P(c_vp), P(Params), c_vp, c_vp, c_vp, c_i64, c_i64, c_vp]),
    ("rsos_sweep", c_i32, [c_vp, c_i64]),
    ("rsos_width", c_i32, [c_vp, P(Width)]),
    ("rsos_log", c_i32, [c_vp, c_i64, c_i64, P(Width)]),
    ("rsos_heights", c_i32, [c_vp, c_vp, ctypes.c_int]),
    ("rsos_moments", c_i32, [c_vp, P(Moments)]),
    ("rsos_time", c_i32, [c_vp, P(c_i64), P(c_vp)]),
    ("rsos_timing", c_i32, [c_vp, ctypes.c_int]),
    ("rsos_timing_read", c_i32, [c_vp, P(c_i64), P(ctypes.c_double), P(ctypes.c_double)]),
    ("rsos_kernel_name", c_i32, [c_vp, ctypes.c_char_p, c_i32]),
    ("rsos_free", c_i32, [c_vp]),
    ("rsos_sweep_static", c_i32, [P(Params), c_vp, c_vp, c_i64, c_i64, c_i64, c_i64, c_vp, c_vp]),
    ("rsos_ms_init", c_i32, [P(c_vp), P(Params), c_i32, c_vp, c_i64, c_vp]),
    ("rsos_ms_sweep", c_i32, [c_vp, c_i64]),
    ("rsos_ms_width", c_i32, [c_vp, P(Width)]),
    ("rsos_ms_log", c_i32, [c_vp, c_i32, c_i64, c_i64, P(Width)]),
    ("rsos_ms_heights", c_i32, [c_vp, c_i32, c_vp]),
    ("rsos_ms_free", c_i32, [c_vp]),
    ("rsos_batch_init", c_i32, [P(c_vp), c_i32, P(Params), c_vp, c_vp, P(c_i64), c_i64, c_vp]),
    ("rsos_batch_sweep", c_i32, [c_vp, P(c_i64), c_i64]),
    ("rsos_batch_width", c_i32, [c_vp, P(Width)]),
    ("rsos_batch_log", c_i32, [c_vp, c_i32, c_i64, c_i64, P(Width)]),
    ("rsos_batch_moments", c_i32, [c_vp, c_i32, P(Moments)]),
    ("rsos_batch_heights", c_i32, [c_vp, c_i32, c_vp, ctypes.c_int]),
    ("rsos_batch_free", c_i32, [c_vp]),
    ("rsos_engine_create", c_i32, [P(c_vp), c_vp, c_i64, c_i32, c_i32, c_vp]),
    ("rsos_engine_submit", c_i32, [c_vp, P(Params), c_i64, P(c_i64), c_i32, c_i32, P(c_i64)]),
    ("rsos_engine_step", c_i32, [c_vp, c_i64, P(c_i32)]),
    ("rsos_engine_poll", c_i32, [c_vp, c_i64, P(c_i32), P(c_i64)]),
    ("rsos_engine_result", c_i32, [c_vp, c_i64, P(Width), c_vp, P(ctypes.c_double)]),
    ("rsos_engine_cancel", c_i32, [c_vp, c_i64]),
    ("rsos_engine_release", c_i32, [c_vp, c_i64]),
    ("rsos_engine_stats", c_i32, [c_vp, P(c_i64)]),
    ("rsos_engine_tune", c_i32, [c_vp, c_i32]),
    ("rsos_engine_destroy", c_i32, [c_vp]),
    ("rsos_tune", c_i32, [P(Params), c_i32, P(Tune)]),
    ("rsos_tune_candidates", c_i32, [P(Params), c_i32, P(Tune), c_i32, P(c_i32)]),
    ("rsos_tune_set", c_i32, [P(Params), c_i32, P(Tune)]),
    ("rsos_tune_clear", c_i32, []),
    ("rsos_tune_save", c_i32, [ctypes.c_char_p]),
    ("rsos_tune_load", c_i32, [ctypes.c_char_p]),
    ("rsos_philox4x32_10", None, [P(c_u32), P(c_u32), P(c_u32)]),
    ("rsos_w2", ctypes.c_double, [c_i32, c_i64, c_i64]),
    ("rsos_strerror", ctypes.c_char_p, [c_i32]),
    ("rsos_last_error", ctypes.c_char_p, []),
    ("rsos_version", ctypes.c_char_p, []),
    ("rsos_debug_fail", c_i32, [c_i32]),
]

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise ImportError(f"{SO_PATH} is missing: run paper_1605_02620_amd/build.py "
                              "(or __graft_entry__.build()) first")
        L = ctypes.CDLL(SO_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != OK:
        msg = lib().rsos_last_error().decode(errors="replace")
        raise RsosError(status, msg)
    return status
