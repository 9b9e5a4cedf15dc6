"""GPU test of rsos_sweep_static, the entry point for callers that cannot
allocate: called through the C ABI on caller tensors, it must give the same
heights and per-sweep records as rsos_init / rsos_sweep / rsos_log on the
same inputs, on two calls in a row (the second on a smaller lattice, so the
shared scratch array keeps the first call's contents), for the block path,
the LDS path and the double-tiling schedule, and across a continuation."""
import ctypes
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[no-alloc] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rsos():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1605_02620_amd as pkg
    return pkg


def _static(L, N, D, seed, h0, t0, s1, s2, n, schedule="checkerboard", stream=None):
    import torch
    from paper_1605_02620_amd import _lib
    from paper_1605_02620_amd.surface import _params
    dev = torch.device("cuda")
    bufs = [torch.zeros(L * L, dtype=torch.int32, device=dev) for _ in range(2)]
    bufs[t0 & 1].copy_(torch.from_numpy(h0.astype(np.int32)))
    log = torch.zeros(max(3 * n, 1), dtype=torch.int64, device=dev)
    p = _params(L, N, D, seed, schedule=schedule)
    st = stream if stream is not None else torch.cuda.current_stream()
    torch.cuda.synchronize()
    _lib.check(_lib.lib().rsos_sweep_static(ctypes.byref(p), ctypes.c_void_p(bufs[0].data_ptr()),
                                            ctypes.c_void_p(bufs[1].data_ptr()), int(t0), int(s1), int(s2),
                                            int(n), ctypes.c_void_p(log.data_ptr()),
                                            ctypes.c_void_p(st.cuda_stream)))
    torch.cuda.synchronize()
    return bufs[(t0 + n) & 1].cpu().numpy(), log.cpu().numpy().reshape(-1, 3)[:n]


def _reference(rsos, L, N, D, seed, h0, t0, n, schedule="checkerboard"):
    s = rsos.Surface(L, N=N, seed=seed, D=D, h0=h0, t0=t0, schedule=schedule)
    s.sweep(n)
    lg = s.log(t0 + 1, n)
    h = s.heights()
    s.close()
    return h, np.stack([lg["s1"], lg["s2"], lg["accepted"]], axis=1)


# (L, N, D, seed, t0, n, start, schedule) -- pairs: each larger call is
# followed by a smaller one
CASES = [
    (2048, 1, 8, 5, 0, 24, "flat", "checkerboard"),
    (512, 3, 8, 6, 7, 9, "rough", "checkerboard"),
    (1024, 2, 16, 7, 0, 6, "rough", "checkerboard"),
    (96, 1, 8, 8, 3, 11, "rough", "checkerboard"),       # LDS path
    (1024, 1, 8, 9, 0, 5, "flat", "double"),
    (256, 4, 8, 10, 2, 4, "cone", "checkerboard"),       # int16 sub-blocks
]


def _h0(L, N, seed, start):
    if start == "flat":
        return workloads.flat(L)
    if start == "cone":
        return workloads.cone(L, N, height=N * L // 4, seed=seed)
    return workloads.rough(L, min(N, 4), seed=seed)


def test_static_matches_handle_path(rsos):
    for (L, N, D, seed, t0, n, start, schedule) in CASES:
        _say(f"L={L} N={N} D={D} seed={seed} t0={t0} n={n} {start} {schedule}")
        h0 = _h0(L, N, seed, start)
        s1 = int(h0.astype(np.int64).sum())
        s2 = int((h0.astype(np.int64) ** 2).sum())
        g_h, g_log = _static(L, N, D, seed, h0, t0, s1, s2, n, schedule)
        r_h, r_log = _reference(rsos, L, N, D, seed, h0, t0, n, schedule)
        assert np.array_equal(g_log, r_log), "records differ"
        assert np.array_equal(g_h, r_h), "heights differ"


def test_static_continuation(rsos):
    """Two calls of 7 and 9 sweeps equal one run of 16 (the second call
    starts from the first's last record)."""
    L, N, D, seed = 512, 1, 8, 77
    h0 = workloads.flat(L)
    h1, log1 = _static(L, N, D, seed, h0, 0, 0, 0, 7)
    h2, log2 = _static(L, N, D, seed, h1, 7, int(log1[-1, 0]), int(log1[-1, 1]), 9)
    r_h, r_log = _reference(rsos, L, N, D, seed, h0, 0, 16)
    assert np.array_equal(np.concatenate([log1, log2]), r_log)
    assert np.array_equal(h2, r_h)


def test_static_rejects_bad_calls(rsos):
    import torch
    from paper_1605_02620_amd import _lib
    from paper_1605_02620_amd.surface import _params
    L = 256
    b = [torch.zeros(L * L, dtype=torch.int32, device="cuda") for _ in range(2)]
    log = torch.zeros(3 * (_lib.STATIC_MAX_SWEEPS + 1), dtype=torch.int64, device="cuda")
    f = _lib.lib().rsos_sweep_static

    def call(p, n, t0=0, s1=0, s2=0):
        return f(ctypes.byref(p), ctypes.c_void_p(b[0].data_ptr()), ctypes.c_void_p(b[1].data_ptr()), t0, s1, s2,
                 n, ctypes.c_void_p(log.data_ptr()), None)
    assert call(_params(L, 1, 8, 1), _lib.STATIC_MAX_SWEEPS + 1) == _lib.E_INVAL
    assert b"outside" in _lib.lib().rsos_last_error()
    assert call(_params(L, 1, 8, 1, packed=True), 1) == _lib.E_INVAL
    assert call(_params(L, 1, 8, 1), 1, s1=5, s2=0) == _lib.E_INVAL
    assert call(_params(L, 1, 8, 1), 0) == _lib.OK
