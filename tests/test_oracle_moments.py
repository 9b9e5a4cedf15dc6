"""Pins of the oracle's height-distribution moments (Eqs. (13)-(15)).

The oracle sums (h - R)^k exactly in 128-bit integers and forms the central
moments as exact rationals.  Pinned against a library routine (scipy's
central moments), the closed-form moments of a two-valued distribution
(at small and at near-2^30 scale, where the 128-bit sums matter), shift
invariance, and the steady-state shape of the RSOS height distribution
(Sec. III.C: |S_h| = 0.270(5), Q_h = 0.15(1); the width distribution's
S = 1.70(1)) at a small size.
"""
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

import workloads


def _phi_float(m):
    return [float(x) for x in m["phi"]]


@pytest.mark.parametrize("L,N,seed,base", [(32, 1, 1, 0), (64, 3, 2, 17), (48, 7, 3, 1 << 20), (128, 2, 4, 5)])
def test_central_moments_match_scipy(oracle, L, N, seed, base):
    h = workloads.rough(L, N, seed=seed, base=base)
    m = oracle.moments(h, L)
    got = _phi_float(m)
    want = [stats.moment(h.astype(np.float64), k) for k in (2, 3, 4)]
    for g, w in zip(got, want):
        assert abs(g - w) <= 1e-9 * max(1.0, abs(w))
    assert m["ref"] == int(h.astype(np.int64).sum()) // (L * L)


@pytest.mark.parametrize("L,ones,scale", [(8, 1, 1), (8, 20, 1), (16, 128, 1), (16, 37, (1 << 30) - 1),
                                          (32, 1000, (1 << 30) - 1)])
def test_two_valued_closed_form(oracle, L, ones, scale):
    """h in {0, M}, a fraction p at M: Phi_2 = M^2 p q, Phi_3 = M^3 p q (q - p),
    Phi_4 = M^4 p q (1 - 3 p q) with q = 1 - p (Bernoulli moments)."""
    rng = np.random.default_rng(ones)
    h = np.zeros(L * L, dtype=np.int32)
    h[rng.choice(L * L, size=ones, replace=False)] = scale
    p = Fraction(ones, L * L)
    q = 1 - p
    M = Fraction(scale)
    want = (M ** 2 * p * q, M ** 3 * p * q * (q - p), M ** 4 * p * q * (1 - 3 * p * q))
    assert oracle.moments(h, L)["phi"] == want


def test_shift_invariance(oracle):
    h = workloads.rough(64, 4, seed=9)
    a = oracle.moments(h, 64)
    for c in (1, 12345, (1 << 29) - 77):
        b = oracle.moments(h + np.int32(c), 64)
        assert b["phi"] == a["phi"]
        assert b["ref"] == a["ref"] + c
        assert b["c"] == a["c"]


def test_power_sums_about_any_reference(oracle):
    """C_k about R and about R' are related by the binomial shift."""
    h = workloads.rough(32, 2, seed=5, base=100)
    a = oracle.power_sums(h, 32, 100)
    b = oracle.power_sums(h, 32, 90)
    n = 32 * 32
    ca = [n] + a
    # sum (h - 90)^k = sum ((h - 100) + 10)^k
    from math import comb
    for k in range(1, 5):
        assert b[k - 1] == sum(comb(k, j) * ca[j] * 10 ** (k - j) for j in range(k + 1))


def test_steady_state_shape(oracle):
    """RSOS at L = 16, N = 1, D = 8 in the steady state (t >= 1000 >> t_x):
    the height distribution has |S_h| near 0.27 (negative: the RSOS
    nonlinearity has negative sign) and Q_h near 0.15; the width
    distribution is right-skewed with S near 1.7."""
    L = 16
    phis, w2 = [], []
    for sd in range(8):
        h = workloads.flat(L)
        oracle.run(h, L, 1, 8, seed=100 + sd, t0=0, n=1000, log=False)
        t = 1000
        for _ in range(2000):
            oracle.run(h, L, 1, 8, seed=100 + sd, t0=t, n=20, log=False)
            t += 20
            phis.append(_phi_float(oracle.moments(h, L)))
            s1, s2 = oracle.sums(h, L)
            w2.append(oracle.width2(L, s1, s2))
    p2, p3, p4 = np.mean(np.array(phis), axis=0)
    s_h = p3 / p2 ** 1.5
    q_h = p4 / p2 ** 2 - 3
    s_w = stats.skew(np.array(w2))
    assert -0.32 <= s_h <= -0.20, s_h
    assert 0.05 <= q_h <= 0.22, q_h
    assert 1.4 <= s_w <= 2.1, s_w
