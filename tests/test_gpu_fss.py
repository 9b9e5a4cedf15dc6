"""The steady-state finite-size-scaling workload (Sec. III.B-C) on the GPU.

A reduced version (L = 32, 64, 128; 32 realizations each) of the paper's
steady-state study: the calibration of Eq. (7), W_sat(L) and its direct fit,
and the width and height distribution shapes in the steady state.  The
physics checks are statistical, with tolerances wide enough for this sample
size; the trajectories themselves are checked bit for bit against the
oracle on one realization per size.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[fss] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fss():
    import torch
    assert torch.cuda.is_available()
    from paper_1605_02620_amd import fss as f
    return f


def test_calibration(fss):
    c = fss.calibrate(1, realizations=8)
    _say(f"calibration {c}")
    assert c["a"] > 0 and c["b"] > 0
    assert 0.15 <= c["beta"] <= 0.3
    assert 0.3 <= c["alpha"] <= 0.45
    assert 100 < fss.t_steady(64, **c) < 20000


def test_steady_state_workload(fss, oracle):
    res = fss.run(sizes=(32, 64, 128), N=1, realizations=32, start=2.0, window=16.0, moment_samples=32)
    _say(f"alpha_fit {res['alpha_fit']:.4f} alpha_eff {res['alpha_eff']} rate {res['attempts_per_ns']:.2f}/ns")
    for L, r in res["sizes"].items():
        _say(f"L={L} {({k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()})}")
    w = [res["sizes"][L]["W_sat"] for L in (32, 64, 128)]
    assert w[0] < w[1] < w[2]
    assert 0.33 <= res["alpha_fit"] <= 0.45
    for L in (32, 64, 128):
        r = res["sizes"][L]
        assert -0.36 <= r["S_h"] <= -0.15, r
        assert -0.05 <= r["Q_h"] <= 0.35, r
        assert 1.0 <= r["S_w2"] <= 2.6, r
    # one realization per size against the oracle, bit for bit at t_end
    oracle.set_threads(16)
    try:
        for L in (32, 64, 128):
            f = next(x for x in res["final"] if x["L"] == L)
            h = workloads.flat(L)
            lg = oracle.run(h, L, 1, 8, seed=f["seed"], t0=0, n=f["t"])
            assert (int(lg[-1, 1]), int(lg[-1, 2])) == (f["s1"], f["s2"]), L
    finally:
        oracle.set_threads(0)
