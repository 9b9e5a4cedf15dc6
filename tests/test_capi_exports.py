"""The C-ABI library loads without a GPU and exports every declared symbol.

No compute call is made here: only the library's load, its symbol table
against include/*.h, the host-side utilities, and the Python binding's
declarations.
"""
import ctypes
import glob
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SO = os.path.join(ROOT, "paper_1605_02620_amd", "librsos.so")


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", " ", txt, flags=re.S)
        for m in re.finditer(r"\b(rsos_\w+)\s*\(", txt):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(SO):
        from paper_1605_02620_amd import build
        build.build(force=True)
    return SO


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("rsos_init", "rsos_sweep", "rsos_width", "rsos_batch_init",
                     "rsos_batch_sweep", "rsos_engine_create", "rsos_engine_submit"):
        assert required in names


def test_every_declared_symbol_is_exported(so):
    out = subprocess.check_output(["nm", "-D", "--defined-only", so], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = sorted(_declared() - exported)
    assert not missing, f"declared but not exported: {missing}"


def test_library_loads_and_binding_matches(so):
    lib = ctypes.CDLL(so)
    from paper_1605_02620_amd import _lib
    declared = _declared()
    bound = {name for name, _, _ in _lib.SIGNATURES}
    assert bound == declared, (sorted(declared - bound), sorted(bound - declared))
    for name in bound:
        getattr(lib, name)
    assert _lib.lib().rsos_version().startswith(b"rsos")


def test_host_philox_matches_oracle(so, oracle):
    """The library's own Philox (the code the kernels use, compiled for the
    host here) against the oracle's independent implementation."""
    from paper_1605_02620_amd import surface
    rng = np.random.default_rng(9)
    for _ in range(300):
        c = [int(v) for v in rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)]
        k = [int(v) for v in rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)]
        assert list(surface.philox(c, k)) == list(oracle.philox(c, k))


def test_host_philox_matches_rocrand(so, rocrand_philox):
    from paper_1605_02620_amd import surface
    for c, k in [([0, 0, 0, 0], [0, 0]), ([5, 6, 7, 8], [9, 10]),
                 ([0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF], [0xFFFFFFFF, 0xFFFFFFFF])]:
        assert list(surface.philox(c, k)) == list(rocrand_philox(c, k))


def test_width_helper(so, oracle):
    from paper_1605_02620_amd import surface
    for (L, s1, s2) in [(2, 3, 9), (64, 12345, 2400000), (16384, 268435456 * 7, 268435456 * 60)]:
        assert surface.w2(L, s1, s2) == oracle.width2(L, s1, s2)


def test_status_strings(so):
    from paper_1605_02620_amd import _lib
    for st in range(-7, 1):
        assert _lib.lib().rsos_strerror(st)


def test_parameter_checks_without_gpu(so):
    """rsos_init validates its parameters on the host before any device call:
    unknown flags, the limits of the 16-bit storage mode (N*L <= 32766, the
    tile-block path, N*D <= 96) and of the double-tiling schedule."""
    from paper_1605_02620_amd import _lib
    lib = _lib.lib()

    def init(L, N, D, flags):
        p = _lib.Params(L, N, D, flags, 1)
        h = ctypes.c_void_p()
        st = lib.rsos_init(ctypes.byref(h), ctypes.byref(p), None, None, None, 0, 0, None)
        return st, lib.rsos_last_error().decode()

    assert init(1024, 1, 8, 8)[0] == _lib.E_INVAL
    assert "flags" in init(1024, 1, 8, 8)[1]
    st, msg = init(1024, 1, 4, _lib.FLAG_DT4)                # double tiling: D = 8 or 16
    assert st == _lib.E_INVAL and "double tiling" in msg
    st, msg = init(1024, 1, 8, _lib.FLAG_DT4 | _lib.FLAG_PACKED16)
    assert st == _lib.E_INVAL and "double-tiling" in msg
    for (L, N, D) in [(1024, 1, 8), (64, 1, 8), (512, 3, 16)]:
        st, msg = init(L, N, D, _lib.FLAG_DT4)
        assert st == _lib.E_INVAL and "d_h" in msg, (L, N, D, msg)
    st, msg = init(16384, 2, 8, _lib.FLAG_PACKED16)          # N L = 32768
    assert st == _lib.E_INVAL and "32766" in msg
    st, msg = init(64, 1, 8, _lib.FLAG_PACKED16)             # LDS-path size
    assert st == _lib.E_INVAL and "LDS" in msg
    st, msg = init(1024, 13, 8, _lib.FLAG_PACKED16)          # N D = 104 > 96
    assert st == _lib.E_INVAL and "tile-block" in msg
    # valid parameters get as far as the NULL buffer check
    for (L, N, D) in [(16384, 1, 8), (8192, 3, 8), (4096, 7, 8), (1024, 12, 8), (256, 1, 8), (512, 3, 16),
                      (256, 1, 2), (256, 2, 4), (256, 2, 32)]:
        st, msg = init(L, N, D, _lib.FLAG_PACKED16)
        assert st == _lib.E_INVAL and "d_h" in msg, (L, N, D, msg)
    # the tile sides: 2, 4, 8, 16, 32; L a multiple of 2 D
    for (L, D) in [(64, 32), (192, 32), (65536, 32), (4, 2)]:
        st, msg = init(L, 1, D, 0)
        assert st == _lib.E_INVAL and "d_h" in msg, (L, D, msg)
    for (L, D) in [(64, 3), (64, 64), (96, 32), (32, 32), (131072, 8)]:
        st, msg = init(L, 1, D, 0)
        assert st == _lib.E_INVAL and ("D=" in msg or "L=" in msg), (L, D, msg)
