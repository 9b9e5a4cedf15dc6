"""GPU parity of the double-tiling schedule (RSOS_FLAG_DT4) against the
oracle's double-tiling sweep, bit for bit, and the domain-size sensitivity
of the steady state (Sec. III.D: 16 x 16 domains against 8 x 8).
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[dt] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rsos():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1605_02620_amd as pkg
    return pkg


def _oracle_dt(oracle, h0, L, N, D, seed, t0, n):
    oracle.set_threads(16)
    try:
        h = h0.copy()
        lg = oracle.run_dt(h, L, N, D, seed=seed, t0=t0, n=n)
    finally:
        oracle.set_threads(0)
    return h, lg


def _compare(g_log, r_log, g_h, r_h):
    for k, name in ((1, "s1"), (2, "s2"), (3, "accepted")):
        bad = np.nonzero(g_log[name] != r_log[:, k])[0]
        assert bad.size == 0, f"{name} differs first at t={int(r_log[bad[0], 0])}"
    assert np.array_equal(g_h, r_h), f"heights differ at {int((g_h != r_h).sum())} sites"


CASES = [
    # L, N, D, seed, sweeps, start
    (64, 1, 8, 1, 200, "flat"),       # LDS-resident
    (128, 2, 16, 2, 60, "rough"),     # LDS-resident, D = 16
    (256, 1, 8, 3, 40, "flat"),       # 16x8 sub-tile blocks
    (384, 2, 8, 4, 20, "rough"),      # T = 48
    (512, 1, 8, 5, 30, "flat"),       # 32x8 sub-tile blocks, int8 staging
    (1024, 3, 8, 6, 12, "rough"),
    (512, 2, 16, 7, 16, "rough"),     # D = 16 blocks
    (256, 2 ** 31 - 1, 8, 8, 6, "flat"),  # no restriction: int32 staging
    (2048, 1, 8, 9, 70, "flat"),      # hipGraph replays
]


@pytest.mark.parametrize("L,N,D,seed,sweeps,start", CASES)
def test_dt_matches_oracle(rsos, oracle, L, N, D, seed, sweeps, start):
    _say(f"L={L} N={N} D={D} seed={seed} sweeps={sweeps} start={start}")
    h0 = workloads.flat(L) if start == "flat" else workloads.rough(L, min(N, 4), seed=seed)
    s = rsos.Surface(L, N=N, seed=seed, D=D, h0=None if start == "flat" else h0, schedule="double")
    if L > 128:
        assert s.kernel_name().endswith(",1>")
    s.sweep(sweeps)
    r_h, r_log = _oracle_dt(oracle, h0, L, N, D, seed, 0, sweeps)
    _compare(s.log(1, sweeps), r_log, s.heights(), r_h)
    s.close()


def test_dt_cone_fallback(rsos, oracle):
    L, N = 1024, 2
    _say("dt cone")
    h0 = workloads.cone(L, N, 900, seed=5)
    s = rsos.Surface(L, N=N, seed=31, D=8, h0=h0, schedule="double")
    s.sweep(6)
    r_h, r_log = _oracle_dt(oracle, h0, L, N, 8, 31, 0, 6)
    _compare(s.log(1, 6), r_log, s.heights(), r_h)


def test_dt_resume_and_batch(rsos, oracle):
    L, N, D, seed = 256, 2, 8, 44
    _say("dt resume and batch")
    h0 = workloads.rough(L, N, seed=1)
    mid, _ = _oracle_dt(oracle, h0, L, N, D, seed, 0, 21)
    s = rsos.Surface(L, N=N, seed=seed, D=D, h0=mid, t0=21, schedule="double")
    s.sweep(7)
    r_h, r_log = _oracle_dt(oracle, mid, L, N, D, seed, 21, 7)
    _compare(s.log(22, 7), r_log, s.heights(), r_h)
    specs = [(256, 1, 5), (512, 2, 6), (64, 1, 7)]
    b = rsos.Batch(specs, D=8, schedule="double")
    b.sweep(9)
    for i, (Lb, Nb, sd) in enumerate(specs):
        r_h, r_log = _oracle_dt(oracle, workloads.flat(Lb), Lb, Nb, 8, sd, 0, 9)
        _compare(b.log(i, 1, 9), r_log, b.heights(i), r_h)


def test_dt_full_size_first_sweeps(rsos, oracle):
    cfg = workloads.cfg_single()
    L, N, D, seed = cfg.L, cfg.N, cfg.D, cfg.seed
    _say(f"dt full size L={L}")
    s = rsos.Surface(L, N=N, seed=seed, D=D, schedule="double")
    s.sweep(2)
    g_log, g_h = s.log(1, 2), s.heights()
    s.close()
    r_h, r_log = _oracle_dt(oracle, workloads.flat(L), L, N, D, seed, 0, 2)
    _compare(g_log, r_log, g_h, r_h)


def test_dt_invalid(rsos):
    from paper_1605_02620_amd._lib import RsosError, E_INVAL
    for kw in ({"D": 4}, {"packed": True}):
        with pytest.raises(RsosError) as e:
            rsos.Surface(512, N=1, schedule="double", **kw)
        assert e.value.status == E_INVAL


def test_domain_size_sensitivity(rsos):
    """Sec. III.D: the steady state with 16 x 16 domains agrees with 8 x 8
    ones (the paper found the finite-size scaling unchanged)."""
    from paper_1605_02620_amd import fss
    res = {}
    for D in (8, 16):
        r = fss.run(sizes=(32, 64, 128), N=1, realizations=32, D=D, start=2.0, window=8.0,
                    moment_samples=8)
        res[D] = r
        _say(f"D={D} alpha_fit {r['alpha_fit']:.4f} W_sat "
             f"{[round(r['sizes'][L]['W_sat'], 4) for L in (32, 64, 128)]}")
    assert abs(res[8]["alpha_fit"] - res[16]["alpha_fit"]) < 0.05
    for D in (8, 16):
        assert 0.33 <= res[D]["alpha_fit"] <= 0.45
