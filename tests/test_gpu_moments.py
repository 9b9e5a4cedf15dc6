"""GPU height-distribution moments (rsos_moments) against the oracle.

The exact power sums about floor(mean) must equal the oracle's 128-bit sums
bit for bit on the same states (the oracle runs the same sweeps itself), for
both storages, the LDS-resident path, batches, and spreads wide enough that
the 128-bit slow path of the kernel runs; central moments agree to rounding.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[moments] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rsos():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1605_02620_amd as pkg
    return pkg


def _oracle_state(oracle, h0, L, N, D, seed, n):
    oracle.set_threads(16)
    try:
        h = h0.copy()
        if n:
            oracle.run(h, L, N, D, seed=seed, t0=0, n=n, log=False)
    finally:
        oracle.set_threads(0)
    return h


def _check(g, oracle, h, L):
    r = oracle.moments(h, L)
    assert g["ref"] == r["ref"]
    assert [g["c1"], g["c2"], g["c3"], g["c4"]] == r["c"]
    for got, want in zip((g["phi2"], g["phi3"], g["phi4"]), r["phi"]):
        w = float(want)
        assert abs(got - w) <= 1e-12 * max(1.0, abs(w)), (got, w)


CASES = [
    # L, N, D, seed, sweeps, start, packed
    (64, 1, 8, 1, 300, "flat", False),        # LDS-resident path
    (256, 1, 8, 7, 0, "flat", False),         # all zero
    (256, 2, 8, 8, 25, "rough", False),
    (512, 1, 8, 9, 40, "flat", True),
    (1024, 4, 8, 10, 10, "rough", True),
    (2048, 12, 8, 11, 3, "cone", False),      # |h - ref| up to ~20000: 128-bit path
    (2048, 12, 8, 11, 3, "cone", True),
    (384, 2, 16, 12, 15, "rough", False),
]


@pytest.mark.parametrize("L,N,D,seed,sweeps,start,packed", CASES)
def test_moments_match_oracle(rsos, oracle, L, N, D, seed, sweeps, start, packed):
    _say(f"L={L} N={N} D={D} sweeps={sweeps} start={start} packed={packed}")
    if start == "flat":
        h0 = workloads.flat(L)
    elif start == "rough":
        h0 = workloads.rough(L, N, seed=seed, base=1000)
    else:
        h0 = workloads.cone(L, N, N * L, seed=seed)
    s = rsos.Surface(L, N=N, seed=seed, D=D, h0=None if start == "flat" else h0, packed=packed)
    s.sweep(sweeps)
    g = s.moments()
    assert g["t"] == sweeps
    _check(g, oracle, _oracle_state(oracle, h0, L, N, D, seed, sweeps), L)
    s.close()


def test_batch_moments(rsos, oracle):
    specs = [(256, 1, 5), (512, 2, 6), (64, 1, 7)]
    _say(f"batch {specs}")
    b = rsos.Batch(specs, D=8)
    b.sweep(12)
    for i, (L, N, seed) in enumerate(specs):
        _check(b.moments(i), oracle, _oracle_state(oracle, workloads.flat(L), L, N, 8, seed, 12), L)


def test_full_size_moments(rsos, oracle):
    """The 16384^2 surface: moments after its first three sweeps against the
    oracle; after 2000 sweeps against the power sums of the returned heights
    (both storages give the same sums)."""
    cfg = workloads.cfg_single()
    L, N, D, seed = cfg.L, cfg.N, cfg.D, cfg.seed
    _say(f"full size L={L}")
    s = rsos.Surface(L, N=N, seed=seed, D=D)
    s.sweep(3)
    _check(s.moments(), oracle, _oracle_state(oracle, workloads.flat(L), L, N, D, seed, 3), L)
    s.sweep(cfg.sweeps - 3)
    g = s.moments()
    h = s.heights().astype(np.int64)
    x = h - g["ref"]
    assert np.abs(x).max() < 400  # keeps every int64 sum below exactly representable bounds
    assert [g["c1"], g["c2"], g["c3"], g["c4"]] == [int((x ** k).sum()) for k in (1, 2, 3, 4)]
    assert abs(g["phi2"] - s.width()["w2"]) <= 1e-12 * g["phi2"]
    p = rsos.Surface(L, N=N, seed=seed, D=D, packed=True)
    p.sweep(cfg.sweeps)
    assert p.moments() == g
