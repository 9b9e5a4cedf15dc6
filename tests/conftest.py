import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a real MI355X (run with -m gpu)")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.fixture(scope="session")
def oracle():
    from oracle import ref
    ref.build()
    return ref


@pytest.fixture(scope="session")
def rocrand_philox():
    """rocRAND's own Philox4x32-10 engine, called on the host through its
    public header API (compiled here with hipcc, host code only)."""
    import ctypes
    import numpy as np
    src = os.path.join(ROOT, "tests", "helpers", "rocrand_philox_probe.cpp")
    out = os.path.join(tempfile.gettempdir(), f"librocrand_probe_{os.getuid()}.so")
    if not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        hipcc = "/opt/rocm/bin/hipcc"
        if not os.path.exists(hipcc):
            pytest.skip("hipcc not available for the rocRAND probe")
        subprocess.check_call([hipcc, "-O2", "-fPIC", "-shared", "-o", out + ".tmp", src])
        os.replace(out + ".tmp", out)
    lib = ctypes.CDLL(out)
    u32p = ctypes.POINTER(ctypes.c_uint32)

    def call(ctr, key):
        c = np.asarray(ctr, dtype=np.uint32).copy()
        k = np.asarray(key, dtype=np.uint32).copy()
        o = np.zeros(4, dtype=np.uint32)
        lib.rocrand_philox_block(c.ctypes.data_as(u32p), k.ctypes.data_as(u32p),
                                 o.ctypes.data_as(u32p))
        return o
    return call
