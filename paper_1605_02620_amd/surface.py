"""Python front end of the single-surface and batched paths.

Argument marshalling only: torch allocates the device buffers and supplies
the stream; every step of a sweep runs in librsos.so's kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import Moments, Params, Tune, Width, check, lib

LOG_DTYPE = np.dtype([("t", np.int64), ("s1", np.int64), ("s2", np.int64),
                      ("accepted", np.int64), ("w2", np.float64)])


def _require_gpu(device):
    dev = torch.device(device)
    if dev.type != "cuda" or not torch.cuda.is_available():
        raise RuntimeError("the RSOS sweep runs only on a ROCm GPU (no CPU fallback)")
    return dev


def _stream_handle(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


SCHEDULES = {"checkerboard": 0, "double": _lib.FLAG_DT4}


def _params(L, N, D, seed, packed=False, schedule="checkerboard", tune=False):
    if schedule not in SCHEDULES:
        raise ValueError(f"schedule must be one of {sorted(SCHEDULES)}")
    flags = (_lib.FLAG_PACKED16 if packed else 0) | SCHEDULES[schedule] | (_lib.FLAG_TUNE if tune else 0)
    return Params(int(L), int(N), int(D), flags, ctypes.c_uint64(int(seed) & (2 ** 64 - 1)).value)


def _widths(buf, n):
    return np.frombuffer(ctypes.string_at(ctypes.addressof(buf), ctypes.sizeof(Width) * n),
                         dtype=LOG_DTYPE).copy()


class Surface:
    """One L x L surface (rsos_init / rsos_sweep / rsos_width).

    packed=True keeps the heights as 16-bit residues in device memory
    (RSOS_FLAG_PACKED16; N*L <= 32766): identical results, half the bytes
    per sweep.  The two int32[L*L] tensors are then the residue pair and
    the int32 readout scratch.

    schedule="double" runs the paper's double-tiling schedule (RSOS_FLAG_DT4)
    instead of the tile checkerboard.

    tune=True takes the launch configuration from the autotuner
    (RSOS_FLAG_TUNE; tuned on first use of the key): same results."""

    def __init__(self, L: int, N: int = 1, seed: int = 0, D: int = 8, h0=None, t0: int = 0,
                 log_cap: int = 0, device="cuda", stream=None, packed: bool = False,
                 schedule: str = "checkerboard", tune: bool = False):
        dev = _require_gpu(device)
        self.L, self.N, self.D, self.seed = int(L), int(N), int(D), int(seed)
        self.packed = bool(packed)
        self.device = dev
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        n = self.L * self.L
        self.bufs = (torch.empty(n, dtype=torch.int32, device=dev),
                     torch.empty(n, dtype=torch.int32, device=dev))
        self.schedule = schedule
        p = _params(L, N, D, seed, self.packed, schedule, tune)
        h0p = None
        if h0 is not None:
            self._h0 = np.ascontiguousarray(np.asarray(h0, dtype=np.int32).reshape(-1))
            if self._h0.size != n:
                raise ValueError("h0 must have L*L elements")
            h0p = self._h0.ctypes.data_as(ctypes.c_void_p)
        self._h = ctypes.c_void_p()
        check(lib().rsos_init(ctypes.byref(self._h), ctypes.byref(p),
                              ctypes.c_void_p(self.bufs[0].data_ptr()),
                              ctypes.c_void_p(self.bufs[1].data_ptr()), h0p, int(t0), int(log_cap),
                              _stream_handle(self.stream)))

    def sweep(self, n_mcs: int):
        check(lib().rsos_sweep(self._h, int(n_mcs)))
        return self

    def width(self) -> np.void:
        w = Width()
        check(lib().rsos_width(self._h, ctypes.byref(w)))
        return _widths(w, 1)[0]

    def log(self, t_from: int, n: int) -> np.ndarray:
        buf = (Width * max(int(n), 1))()
        check(lib().rsos_log(self._h, int(t_from), int(n), buf))
        return _widths(buf, int(n))

    def time(self) -> int:
        t = ctypes.c_int64()
        check(lib().rsos_time(self._h, ctypes.byref(t), None))
        return t.value

    def heights(self) -> np.ndarray:
        out = np.empty(self.L * self.L, dtype=np.int32)
        check(lib().rsos_heights(self._h, out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def moments(self) -> dict:
        """Height-distribution moments of the current state (rsos_moments):
        exact power sums c1..c4 about ref = floor(mean), central moments
        phi2..phi4."""
        m = Moments()
        check(lib().rsos_moments(self._h, ctypes.byref(m)))
        return m.as_dict()

    def heights_tensor(self) -> torch.Tensor:
        """The current state as an int32 device tensor: a view of one of the
        buffers, or (packed) a new tensor the library converts into."""
        if not self.packed:
            return self.bufs[self.time() & 1]
        out = torch.empty(self.L * self.L, dtype=torch.int32, device=self.device)
        check(lib().rsos_heights(self._h, ctypes.c_void_p(out.data_ptr()), 1))
        return out

    def kernel_name(self) -> str:
        buf = ctypes.create_string_buffer(128)
        check(lib().rsos_kernel_name(self._h, buf, 128))
        return buf.value.decode()

    def timing(self, enable: bool = True):
        """Times every sweep's tile-block kernels with HIP events recorded
        at their start and end (rsos_timing)."""
        check(lib().rsos_timing(self._h, int(bool(enable))))

    def timing_read(self):
        """(launches, mean ms, total ms) of the timed kernel launches."""
        n, m, t = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
        check(lib().rsos_timing_read(self._h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(t)))
        return n.value, m.value, t.value

    def close(self):
        if self._h:
            check(lib().rsos_free(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent surfaces (one D) swept together: one block-kernel
    launch per sweep covers every surface that still has sweeps to do."""

    ALIGN = 64  # elements (256 bytes) between surfaces in the pool

    def __init__(self, specs, D: int = 8, log_cap: int = 0, device="cuda", stream=None,
                 packed: bool = False, schedule: str = "checkerboard", tune: bool = False):
        dev = _require_gpu(device)
        self.specs = [(int(L), int(N), int(seed)) for (L, N, seed) in specs]
        self.D = int(D)
        self.packed = bool(packed)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        offs, off = [], 0
        for (L, _, _) in self.specs:
            offs.append(off)
            off += -(-L * L // self.ALIGN) * self.ALIGN
        self.offsets = np.asarray(offs, dtype=np.int64)
        self.pool = torch.empty(max(off, 1), dtype=torch.int32, device=dev)
        self.work = torch.empty(max(off, 1), dtype=torch.int32, device=dev)
        self.schedule = schedule
        ps = (Params * len(self.specs))(*[_params(L, N, D, s, self.packed, schedule, tune)
                                          for (L, N, s) in self.specs])
        self._h = ctypes.c_void_p()
        check(lib().rsos_batch_init(ctypes.byref(self._h), len(self.specs), ps,
                                    ctypes.c_void_p(self.pool.data_ptr()),
                                    ctypes.c_void_p(self.work.data_ptr()),
                                    self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    int(log_cap), _stream_handle(self.stream)))

    def __len__(self):
        return len(self.specs)

    def sweep(self, n_mcs):
        if np.isscalar(n_mcs):
            check(lib().rsos_batch_sweep(self._h, None, int(n_mcs)))
        else:
            arr = np.ascontiguousarray(n_mcs, dtype=np.int64)
            assert arr.size == len(self.specs)
            check(lib().rsos_batch_sweep(self._h, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 0))
        return self

    def width(self) -> np.ndarray:
        buf = (Width * len(self.specs))()
        check(lib().rsos_batch_width(self._h, buf))
        return _widths(buf, len(self.specs))

    def log(self, i: int, t_from: int, n: int) -> np.ndarray:
        buf = (Width * max(int(n), 1))()
        check(lib().rsos_batch_log(self._h, int(i), int(t_from), int(n), buf))
        return _widths(buf, int(n))

    def moments(self, i: int) -> dict:
        m = Moments()
        check(lib().rsos_batch_moments(self._h, int(i), ctypes.byref(m)))
        return m.as_dict()

    def heights(self, i: int) -> np.ndarray:
        L = self.specs[i][0]
        out = np.empty(L * L, dtype=np.int32)
        check(lib().rsos_batch_heights(self._h, int(i), out.ctypes.data_as(ctypes.c_void_p), 0))
        return out

    def close(self):
        if self._h:
            check(lib().rsos_batch_free(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MultiSurface:
    """Multisurface lock-step mode (rsos_ms_*): `groups` groups of 128
    realizations of one L x L surface; the realizations of a group share
    the sequence of selected sites and apply each selection with
    probability 1/2.  Realization index i = 128 g + r."""

    REAL = 128

    def __init__(self, L: int, N: int = 1, seed: int = 0, groups: int = 1, log_cap: int = 0,
                 device="cuda", stream=None):
        dev = _require_gpu(device)
        self.L, self.N, self.seed, self.groups = int(L), int(N), int(seed), int(groups)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        words = self.groups * self.L * self.L * 64
        self.lat = torch.empty(words, dtype=torch.int32, device=dev)
        p = _params(L, N, 8, seed)
        self._h = ctypes.c_void_p()
        check(lib().rsos_ms_init(ctypes.byref(self._h), ctypes.byref(p), self.groups,
                                 ctypes.c_void_p(self.lat.data_ptr()), int(log_cap),
                                 _stream_handle(self.stream)))

    def __len__(self):
        return self.groups * self.REAL

    def sweep(self, n_mcs: int):
        check(lib().rsos_ms_sweep(self._h, int(n_mcs)))
        return self

    def width(self) -> np.ndarray:
        buf = (Width * len(self))()
        check(lib().rsos_ms_width(self._h, buf))
        return _widths(buf, len(self))

    def log(self, i: int, t_from: int, n: int) -> np.ndarray:
        buf = (Width * max(int(n), 1))()
        check(lib().rsos_ms_log(self._h, int(i), int(t_from), int(n), buf))
        return _widths(buf, int(n))

    def heights(self, i: int) -> np.ndarray:
        out = np.empty(self.L * self.L, dtype=np.int32)
        check(lib().rsos_ms_heights(self._h, int(i), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def close(self):
        if self._h:
            check(lib().rsos_ms_free(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune(L: int, N: int = 1, D: int = 8, batch: bool = False, packed: bool = False,
         schedule: str = "checkerboard") -> dict:
    """The autotuner's configuration for the key (L, N, D, storage,
    schedule, alone or batched), tuning it on first use (rsos_tune)."""
    p = _params(L, N, D, 0, packed, schedule)
    t = Tune()
    check(lib().rsos_tune(ctypes.byref(p), int(bool(batch)), ctypes.byref(t)))
    return t.as_dict()


def tune_candidates(L: int, N: int = 1, D: int = 8, batch: bool = False, packed: bool = False,
                    schedule: str = "checkerboard") -> list:
    """Every launch configuration the autotuner considers for the key."""
    p = _params(L, N, D, 0, packed, schedule)
    n = ctypes.c_int32()
    check(lib().rsos_tune_candidates(ctypes.byref(p), int(bool(batch)), None, 0, ctypes.byref(n)))
    buf = (Tune * max(n.value, 1))()
    check(lib().rsos_tune_candidates(ctypes.byref(p), int(bool(batch)), buf, n.value, ctypes.byref(n)))
    return [buf[i].as_dict() for i in range(n.value)]


def tune_set(L: int, N: int, D: int, choice: dict, batch: bool = False, packed: bool = False,
             schedule: str = "checkerboard"):
    """Enters a configuration for the key without timing it (rsos_tune_set)."""
    p = _params(L, N, D, 0, packed, schedule)
    t = Tune(**{k: choice[k] for k in ("TX", "TY", "NT", "elem", "xmode")},
             graph_sweeps=int(choice.get("graph_sweeps") or 32))
    check(lib().rsos_tune_set(ctypes.byref(p), int(bool(batch)), ctypes.byref(t)))


def tune_clear():
    check(lib().rsos_tune_clear())


def tune_save(path: str):
    check(lib().rsos_tune_save(str(path).encode()))


def tune_load(path: str):
    check(lib().rsos_tune_load(str(path).encode()))


def philox(ctr, key):
    """The library's own Philox4x32-10 block function, run on the host."""
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().rsos_philox4x32_10(c, k, o)
    return np.array(list(o), dtype=np.uint32)


def w2(L, s1, s2):
    return float(lib().rsos_w2(int(L), int(s1), int(s2)))


__all__ = ["Surface", "Batch", "MultiSurface", "philox", "w2", "tune", "tune_candidates", "tune_set",
           "tune_clear", "tune_save", "tune_load", "LOG_DTYPE", "_lib"]
