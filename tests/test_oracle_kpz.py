"""Statistical-physics pins of the oracle: KPZ scaling (Sec. III).

The paper reports beta = 0.241(1) (Sec. III.A, Table I) and
alpha = 0.390(4) (Sec. III.B; direct fit 0.392(1) for N = 1 over
32 <= L <= 512).  Exponents refer to W, so fits of ln W^2 are halved
(Eqs. (3), (4)).  A wrong acceptance rule would leave this class: random
deposition never saturates and grows with beta = 1/2, and a linear (EW)
surface in 2+1 dimensions has alpha = beta = 0 (logarithmic growth).
The tolerances allow for small-size and short-time corrections, which the
paper discusses at length for exactly these lattice sizes (Sec. III.B).
"""
import numpy as np

import workloads


def _w2(oracle, L, lg):
    return np.array([oracle.width2(L, a, b) for a, b in zip(lg[:, 1], lg[:, 2])])


def _beta(ts, w2, lo, hi):
    m = (ts >= lo) & (ts <= hi)
    return np.polyfit(np.log(ts[m]), np.log(w2[m]), 1)[0] / 2


def test_growth_exponent_tiled_and_rs(oracle):
    """W^2 ~ t^(2 beta) (Eq. (3)) in the growth regime: the tiled schedule
    on L = 2048 over 64 <= t <= 1024 (mean of two seeds), random-sequential
    updates on L = 1024 over 32 <= t <= 512."""
    oracle.set_threads(8)
    try:
        L = 2048
        b = []
        for seed in (3, 4):
            h = workloads.flat(L)
            lg = oracle.run(h, L, 1, 8, seed=seed, t0=0, n=1024)
            b.append(_beta(lg[:, 0], _w2(oracle, L, lg), 64, 1024))
        b_tc = float(np.mean(b))
    finally:
        oracle.set_threads(0)
    assert 0.22 <= b_tc <= 0.26, b
    L = 1024
    h = workloads.flat(L)
    lg = oracle.rs_run(h, L, 1, rs_seed=3, t0=0, n=512)
    b_rs = _beta(lg[:, 0], _w2(oracle, L, lg), 32, 512)
    assert 0.22 <= b_rs <= 0.26, b_rs
    # Sec. III.C: the domain decomposition must not change the exponents
    assert abs(b_tc - b_rs) < 0.02, (b, b_rs)


def test_roughness_exponent_tiled(oracle):
    """W_sat^2 ~ L^(2 alpha) (Eq. (12)) over L = 32, 64, 128, time averages
    over 40 t_x after a 3 t_x burn-in, t_x = L^1.6 (z of Sec. III.B)."""
    alphas = []
    for seed in (2, 3):
        ws = []
        for L in (32, 64, 128):
            oracle.set_threads(8 if L >= 128 else 0)
            try:
                tx = L ** 1.6
                burn, n = int(3 * tx), int(40 * tx)
                h = workloads.flat(L)
                lg = oracle.run(h, L, 1, 8, seed=seed, t0=0, n=burn + n)
            finally:
                oracle.set_threads(0)
            ws.append(_w2(oracle, L, lg[burn:]).mean())
        alphas.append(np.polyfit(np.log([32, 64, 128]), np.log(ws), 1)[0] / 2)
    a = float(np.mean(alphas))
    assert 0.36 <= a <= 0.42, alphas
