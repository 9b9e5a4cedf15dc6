"""Exact-enumeration pins of the oracle on tiny lattices.

The full probability distribution over lattice states is propagated attempt
by attempt (oracle/brute.py) and compared, by a chi-square test, with the
frequencies of the C oracle's sampled runs over many seeds.  A dropped
neighbour, a wrong colour, a wrong shift range or a biased site field would
move probability mass between states and fail these tests.  The stationary
<W^2> of small random-sequential lattices is solved exactly from the Markov
chain and compared with long time averages of the plain RS reference.
"""
from collections import Counter

import numpy as np
import pytest
from scipy.stats import chi2 as chi2_dist

import workloads
from oracle import brute


def _tc_counts(oracle, h0, L, N, D, sweeps, nseed):
    counts = Counter()
    for seed in range(nseed):
        h = h0.copy()
        oracle.run(h, L, N, D, seed=seed, t0=0, n=sweeps, log=False)
        counts[tuple(int(v) for v in h)] += 1
    return counts


@pytest.mark.parametrize("start,N", [("flat", 1), ("rough", 1)])
def test_tiled_L4_D2_distribution(oracle, start, N):
    """One sweep on a 4 x 4 torus with 2 x 2 domains: 16 origins, 2 tiles per
    colour, 4 attempts per tile.  The rough start (seed 7) makes rejections
    frequent from the first attempt on."""
    L, D = 4, 2
    h0 = workloads.flat(L) if start == "flat" else workloads.rough(L, N, seed=7)
    exact = brute.tc_distribution(h0, L, N, D, 1)
    assert abs(sum(exact.values()) - 1.0) < 1e-9
    counts = _tc_counts(oracle, h0, L, N, D, 1, 120000)
    stat, dof, unknown = brute.chi2_against(exact, counts)
    assert unknown == 0, "oracle produced a state the exact enumeration cannot reach"
    assert dof > 1000  # most of the mass sits in bins with expected count >= 5
    p = chi2_dist.sf(stat, dof)
    assert p > 1e-4, (stat, dof, p)


def test_rs_L3_distribution(oracle):
    """Random-sequential reference: 9 attempts (one sweep) on a 3 x 3 torus."""
    L, N = 3, 1
    exact = brute.rs_distribution(workloads.flat(L), L, N, L * L)
    counts = Counter()
    for seed in range(60000):
        h = workloads.flat(L)
        oracle.rs_run(h, L, N, rs_seed=seed * 7919 + 1, t0=0, n=1)
        counts[tuple(int(v) for v in h)] += 1
    stat, dof, unknown = brute.chi2_against(exact, counts)
    assert unknown == 0
    assert chi2_dist.sf(stat, dof) > 1e-4, (stat, dof)


def test_exact_stationary_width_L2():
    """The 2 x 2, N = 1 chain has 19 relative-height states; <W^2> = 51/188."""
    from fractions import Fraction
    m, w2 = brute.rs_stationary_w2(2, 1, exact=True)
    assert m == 19
    assert w2 == Fraction(51, 188)


@pytest.mark.parametrize("L,N", [(2, 1), (3, 1), (2, 2)])
def test_rs_stationary_time_average(oracle, L, N):
    m, w2_exact = brute.rs_stationary_w2(L, N)
    h = workloads.flat(L)
    oracle.rs_run(h, L, N, rs_seed=99, t0=0, n=2000)  # burn-in
    log = oracle.rs_run(h, L, N, rs_seed=100, t0=2000, n=200000)
    w = np.array([oracle.width2(L, a, b) for a, b in zip(log[:, 1], log[:, 2])])
    batches = w.reshape(200, -1).mean(axis=1)  # batch means for the standard error
    se = batches.std(ddof=1) / np.sqrt(len(batches))
    assert abs(w.mean() - float(w2_exact)) < 4 * se, (w.mean(), float(w2_exact), se)
