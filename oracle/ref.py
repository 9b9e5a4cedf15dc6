"""ctypes front end of the CPU oracle (oracle/librsos_ref.so).

TEST INFRASTRUCTURE ONLY: the slow, plainly written CPU reference for the
RSOS deposition sweep of Kelling, Odor & Gemming (Sec. II schedule, Sec. I
deposition rule, Eq. (2) width).  Only tests, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the product library and never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "librsos_ref.so")
_SRC = os.path.join(_HERE, "rsos_ref.c")

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_u32p = ctypes.POINTER(ctypes.c_uint32)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over independent tiles)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        L.ref_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.ref_origin.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, _i32p, _i32p]
        L.ref_tile_sites.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                     ctypes.c_uint32, ctypes.c_uint32, _i32p, _i32p]
        L.ref_tile_sites.restype = ctypes.c_int
        L.ref_word_fields.argtypes = [ctypes.c_int, ctypes.c_uint32, _i32p]
        L.ref_word_fields.restype = ctypes.c_int
        L.ref_attempt.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.ref_attempt.restype = ctypes.c_int
        L.ref_rsos_holds.argtypes = [_i32p, ctypes.c_int, ctypes.c_int]
        L.ref_rsos_holds.restype = ctypes.c_int
        L.ref_sums.argtypes = [_i32p, ctypes.c_int, _i64p, _i64p]
        L.ref_power_sums.argtypes = [_i32p, ctypes.c_int, ctypes.c_int64, _i64p]
        L.ref_run_ms.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, _i64p]
        L.ref_run_ms.restype = ctypes.c_int
        L.ref_run_ms_injected.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int64, _i32p, _i32p, _i32p, _i64p]
        L.ref_run_ms_injected.restype = ctypes.c_int
        L.ref_run_dt.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                 ctypes.c_int64, ctypes.c_int64, _i64p]
        L.ref_run_dt.restype = ctypes.c_int
        L.ref_run_dt_injected.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_int64, _i32p, _i32p, _i64p]
        L.ref_run_dt_injected.restype = ctypes.c_int
        L.ref_run.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                              ctypes.c_int64, ctypes.c_int64, _i64p]
        L.ref_run.restype = ctypes.c_int
        L.ref_run_injected.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int64, _i32p, _i32p, _i64p]
        L.ref_run_injected.restype = ctypes.c_int
        L.ref_rs_run.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64,
                                 ctypes.c_int64, ctypes.c_int64, _i64p]
        L.ref_rs_run.restype = ctypes.c_int
        L.ref_rs_injected.argtypes = [_i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int64, _i32p]
        L.ref_rs_injected.restype = ctypes.c_int64
        L.ref_set_threads.argtypes = [ctypes.c_int]
        L.ref_set_tile_order_seed.argtypes = [ctypes.c_uint64]
        _lib = L
    return _lib


def _p32(a):
    return a.ctypes.data_as(_i32p)


def _p64(a):
    return a.ctypes.data_as(_i64p)


class OracleError(RuntimeError):
    pass


def philox(ctr, key):
    """Philox4x32-10 block (SC'11): 4 output words for a 4-word counter, 2-word key."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    o = np.zeros(4, dtype=np.uint32)
    lib().ref_philox4x32_10(c.ctypes.data_as(_u32p), k.ctypes.data_as(_u32p),
                            o.ctypes.data_as(_u32p))
    return o


def origin(D, seed, s):
    ox, oy = ctypes.c_int32(), ctypes.c_int32()
    lib().ref_origin(D, seed, s, ctypes.byref(ox), ctypes.byref(oy))
    return ox.value, oy.value


def word_fields(D, word):
    f = np.zeros(16, dtype=np.int32)
    n = lib().ref_word_fields(D, word, _p32(f))
    if n < 0:
        raise OracleError("bad D")
    return [int(x) for x in f[:n]]


def tile_sites(D, seed, s, p, tile_id):
    u = np.zeros(D * D, dtype=np.int32)
    v = np.zeros(D * D, dtype=np.int32)
    if lib().ref_tile_sites(D, seed, s, p, tile_id, _p32(u), _p32(v)) != 0:
        raise OracleError("bad D")
    return u, v


def set_threads(n: int):
    lib().ref_set_threads(int(n))


def set_tile_order_seed(seed: int):
    lib().ref_set_tile_order_seed(int(seed))


def _check(rc):
    if rc == -1:
        raise OracleError("invalid arguments")
    if rc == -2:
        raise OracleError("initial heights violate the RSOS restriction")
    if rc != 0:
        raise OracleError(f"oracle error {rc}")


def run(h, L, N, D, seed, t0, n, log=True):
    """Tile-checkerboard sweeps t0..t0+n-1 on h (int32[L*L], modified in place).

    Returns the per-sweep log as int64[n, 4] = (t, S1, S2, A) or None."""
    assert h.dtype == np.int32 and h.flags.c_contiguous and h.size == L * L
    lg = np.zeros((max(n, 1), 4), dtype=np.int64) if log else None
    _check(lib().ref_run(_p32(h), L, N, D, seed, t0, n, _p64(lg) if log else None))
    return lg[:n] if log else None


def run_dt(h, L, N, D, seed, t0, n, log=True):
    """Double-tiling sweeps t0..t0+n-1 on h (in place); log as run()."""
    assert h.dtype == np.int32 and h.flags.c_contiguous and h.size == L * L
    lg = np.zeros((max(n, 1), 4), dtype=np.int64) if log else None
    _check(lib().ref_run_dt(_p32(h), L, N, D, seed, t0, n, _p64(lg) if log else None))
    return lg[:n] if log else None


def run_ms(h, L, N, D, seed, t0, n, log=True):
    """Multisurface lock-step sweeps of R realizations; h is int32[R, L*L]
    (modified in place).  Returns int64[R, n, 4] = (t, S1, S2, A) or None."""
    assert h.dtype == np.int32 and h.flags.c_contiguous and h.ndim == 2 and h.shape[1] == L * L
    R = h.shape[0]
    lg = np.zeros((R, max(n, 1), 4), dtype=np.int64) if log else None
    _check(lib().ref_run_ms(_p32(h), R, L, N, D, seed, t0, n, _p64(lg) if log else None))
    return lg[:, :n] if log else None


def run_ms_injected(h, L, N, D, origins, sites, coins):
    """One realization of the lock-step schedule along injected choices."""
    origins = np.ascontiguousarray(origins, dtype=np.int32)
    sites = np.ascontiguousarray(sites, dtype=np.int32)
    coins = np.ascontiguousarray(coins, dtype=np.int32)
    n = origins.shape[0]
    lg = np.zeros((max(n, 1), 4), dtype=np.int64)
    _check(lib().ref_run_ms_injected(_p32(h), L, N, D, n, _p32(origins), _p32(sites), _p32(coins),
                                     _p64(lg)))
    return lg[:n]


def run_dt_injected(h, L, N, D, origins, sites):
    """Double-tiling sweeps driven by injected choices (see rsos_ref.h)."""
    origins = np.ascontiguousarray(origins, dtype=np.int32)
    sites = np.ascontiguousarray(sites, dtype=np.int32)
    n = origins.shape[0]
    lg = np.zeros((max(n, 1), 4), dtype=np.int64)
    _check(lib().ref_run_dt_injected(_p32(h), L, N, D, n, _p32(origins), _p32(sites), _p64(lg)))
    return lg[:n]


def run_injected(h, L, N, D, origins, sites):
    """Sweeps driven by injected choices (see rsos_ref.h)."""
    origins = np.ascontiguousarray(origins, dtype=np.int32)
    sites = np.ascontiguousarray(sites, dtype=np.int32)
    n = origins.shape[0]
    assert sites.size == n * L * L
    lg = np.zeros((max(n, 1), 4), dtype=np.int64)
    _check(lib().ref_run_injected(_p32(h), L, N, D, n, _p32(origins), _p32(sites), _p64(lg)))
    return lg[:n]


def rs_run(h, L, N, rs_seed, t0, n):
    lg = np.zeros((max(n, 1), 4), dtype=np.int64)
    _check(lib().ref_rs_run(_p32(h), L, N, rs_seed, t0, n, _p64(lg)))
    return lg[:n]


def rs_injected(h, L, N, sites):
    sites = np.ascontiguousarray(sites, dtype=np.int32)
    return int(lib().ref_rs_injected(_p32(h), L, N, sites.size // 2, _p32(sites)))


def attempt(h, L, N, x, y):
    return int(lib().ref_attempt(_p32(h), L, N, x, y))


def rsos_holds(h, L, N):
    return bool(lib().ref_rsos_holds(_p32(h), L, N))


def sums(h, L):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    lib().ref_sums(_p32(h), L, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def power_sums(h, L, R):
    """C_k = sum (h - R)^k, k = 1..4, exact (Python ints)."""
    out = np.zeros(8, dtype=np.int64)
    lib().ref_power_sums(_p32(h), L, int(R), _p64(out))
    vals = []
    for k in range(4):
        lo, hi = int(out[2 * k]) & (2 ** 64 - 1), int(out[2 * k + 1])
        vals.append((hi << 64) | lo)
    return vals


def central_moments(n, R, c):
    """Exact central moments Phi_2..Phi_4 of a distribution of n integer
    values (Eqs. (13)-(15), sums over the sites of one surface) from the
    power sums c = (C_1..C_4) about R: with d = mean - R = C_1/n, the binomial
    expansion of (h - R - d)^k."""
    n = int(n)
    m = [Fraction(1)] + [Fraction(int(ck), n) for ck in c]   # raw moments about R
    d = m[1]
    phi2 = m[2] - d * d
    phi3 = m[3] - 3 * d * m[2] + 2 * d ** 3
    phi4 = m[4] - 4 * d * m[3] + 6 * d * d * m[2] - 3 * d ** 4
    return phi2, phi3, phi4


def moments(h, L):
    """Height-distribution moments of one surface: reference R = floor(mean),
    power sums about R, exact central moments (Fractions)."""
    s1, _ = sums(h, L)
    n = int(L) * int(L)
    R = s1 // n
    c = power_sums(h, L, R)
    return {"ref": R, "c": c, "phi": central_moments(n, R, c)}


def width2(L, s1, s2):
    """Eq. (2): W^2 = S2/L^2 - (S1/L^2)^2, evaluated as the exact rational
    (L^2 S2 - S1^2) / L^4 and rounded once to the nearest double."""
    L2 = int(L) * int(L)
    return float(Fraction(L2 * int(s2) - int(s1) * int(s1), L2 * L2))
