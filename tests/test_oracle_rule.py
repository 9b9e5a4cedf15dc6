"""Pins of the oracle's deposition rule, schedule and sums.

Each test checks the C oracle against something other than itself: an
independent pure-Python application of the RSOS rule along the same injected
choices, invariants the model guarantees (the restriction of Sec. I holds at
all times; Eq. (2)'s sums follow from the heights and from the accepted
count), closed forms of unrestricted deposition, and the independence of
the result from the order in which independent domains are updated
(Sec. II: sets of domains updated by independent workers).
"""
import numpy as np
import pytest

import workloads
from oracle import brute

INT32_MAX = 2 ** 31 - 1


@pytest.mark.parametrize("L,D,N,sweeps,start", [
    (4, 2, 1, 3, "flat"), (8, 2, 1, 4, "rough"), (8, 4, 2, 3, "rough"),
    (16, 8, 1, 3, "flat"), (32, 8, 1, 2, "rough"), (32, 16, 3, 2, "rough"),
    (64, 32, 2, 2, "rough"),
])
def test_injected_path_matches_python_rule(oracle, L, D, N, sweeps, start):
    rng = np.random.default_rng(L * 100 + D * 10 + N)
    h0 = workloads.flat(L) if start == "flat" else workloads.rough(L, N, seed=L + D)
    origins = rng.integers(0, 2 * D, size=(sweeps, 2)).astype(np.int32)
    sites = rng.integers(0, D * D, size=sweeps * L * L).astype(np.int32)
    h = h0.copy()
    log = oracle.run_injected(h, L, N, D, origins, sites)
    st, acc = brute.tc_apply_choices(h0, L, N, D, [tuple(o) for o in origins], sites)
    assert tuple(int(v) for v in h) == st
    assert [int(a) for a in log[:, 3]] == acc


def test_rs_injected_matches_python_rule(oracle):
    rng = np.random.default_rng(7)
    for (L, N) in [(3, 1), (5, 2), (8, 1)]:
        h0 = workloads.rough(L, N, seed=L)
        sites = rng.integers(0, L, size=(400, 2)).astype(np.int32)
        h = h0.copy()
        a = oracle.rs_injected(h, L, N, sites.reshape(-1))
        st = tuple(int(v) for v in h0)
        acc = 0
        for (x, y) in sites:
            nxt = brute.deposit(st, L, N, int(x), int(y))
            acc += nxt != st
            st = nxt
        assert tuple(int(v) for v in h) == st and a == acc


def test_single_attempt_rule_by_hand(oracle):
    """Hand-worked cases of the restriction on a 4 x 4 torus, N = 1."""
    L = 4
    h = np.zeros(16, dtype=np.int32)
    assert oracle.attempt(h, L, 1, 1, 1) == 1 and h[1 * 4 + 1] == 1   # flat: always accepted
    assert oracle.attempt(h, L, 1, 1, 1) == 0 and h[1 * 4 + 1] == 1   # would make a step of 2
    assert oracle.attempt(h, L, 1, 2, 1) == 1                           # neighbour at 1: step 1 ok
    assert oracle.attempt(h, L, 1, 0, 1) == 1                           # the other side
    # periodic wrap: site (3, 0) neighbours (0, 0) across the boundary
    h[:] = 1
    h[0] = 0
    assert oracle.attempt(h, L, 1, 3, 0) == 0   # 2 - 0 > 1 across the x wrap
    assert oracle.attempt(h, L, 1, 0, 3) == 0   # 2 - 0 > 1 across the y wrap
    assert oracle.attempt(h, L, 2, 3, 0) == 1   # allowed with N = 2


@pytest.mark.parametrize("L,N,D", [(32, 1, 8), (64, 2, 8), (48, 1, 4), (64, 4, 16), (128, 2, 32)])
def test_invariants_every_sweep(oracle, L, N, D):
    """RSOS restriction after every sweep; S1(t) = S1(0) + accepted; S1 and S2
    equal sums recomputed from the heights; 0 < A <= L^2."""
    h = workloads.rough(L, N, seed=3)
    s1_0, _ = oracle.sums(h, L)
    total = 0
    for t in range(12):
        log = oracle.run(h, L, N, D, seed=11, t0=t, n=1)
        assert oracle.rsos_holds(h, L, N)
        s1, s2 = oracle.sums(h, L)
        assert (log[0, 1], log[0, 2]) == (s1, s2)
        assert (np.int64(h).sum(), (np.int64(h) ** 2).sum()) == (s1, s2)
        total += int(log[0, 3])
        assert s1 == s1_0 + total
        assert 0 < log[0, 3] <= L * L
        assert log[0, 0] == t + 1


def test_resume_is_exact(oracle):
    L, N, D = 64, 1, 8
    a = workloads.flat(L)
    la = oracle.run(a, L, N, D, seed=5, t0=0, n=10)
    b = workloads.flat(L)
    lb1 = oracle.run(b, L, N, D, seed=5, t0=0, n=4)
    lb2 = oracle.run(b, L, N, D, seed=5, t0=4, n=6)
    assert np.array_equal(a, b)
    assert np.array_equal(la, np.concatenate([lb1, lb2]))


def test_order_and_threads_do_not_matter(oracle):
    L, N, D = 64, 2, 8
    ref_h = workloads.rough(L, N, seed=9)
    base = ref_h.copy()
    lb = oracle.run(base, L, N, D, seed=77, t0=3, n=5)
    try:
        for threads, order in [(1, 0), (4, 0), (1, 12345), (8, 999)]:
            oracle.set_threads(threads)
            oracle.set_tile_order_seed(order)
            h = ref_h.copy()
            lg = oracle.run(h, L, N, D, seed=77, t0=3, n=5)
            assert np.array_equal(h, base) and np.array_equal(lg, lb)
    finally:
        oracle.set_threads(0)
        oracle.set_tile_order_seed(0)


def test_invalid_inputs_rejected(oracle):
    L = 32
    h = workloads.violating(L, 1, seed=1)
    with pytest.raises(oracle.OracleError):
        oracle.run(h, L, 1, 8, seed=0, t0=0, n=1)
    with pytest.raises(oracle.OracleError):
        oracle.run(workloads.flat(24), 24, 1, 8, seed=0, t0=0, n=1)   # L not a multiple of 2D
    with pytest.raises(oracle.OracleError):
        oracle.run(workloads.flat(32), 32, 1, 6, seed=0, t0=0, n=1)   # D not a power of two
    with pytest.raises(oracle.OracleError):
        oracle.run(workloads.flat(32), 32, 0, 8, seed=0, t0=0, n=1)   # N < 1


def test_unrestricted_closed_form_tiled(oracle):
    """N = INT32_MAX accepts every attempt: S1 = t L^2 exactly, and each site
    gets Binomial(D^2, 1/D^2) deposits per sweep, so E[W^2] = t (1 - 1/D^2)."""
    L, t = 64, 6
    for D in (2, 8):
        w2 = []
        for seed in range(40):
            h = workloads.flat(L)
            log = oracle.run(h, L, INT32_MAX, D, seed=seed, t0=0, n=t)
            assert [int(x) for x in log[:, 1]] == [(k + 1) * L * L for k in range(t)]
            assert all(int(a) == L * L for a in log[:, 3])
            w2.append(oracle.width2(L, log[-1, 1], log[-1, 2]))
        w2 = np.asarray(w2)
        expect = float(brute.tiled_rd_w2_mean(t, D))
        se = w2.std(ddof=1) / np.sqrt(len(w2))
        assert abs(w2.mean() - expect) < 4 * se, (D, w2.mean(), expect, se)


def test_unrestricted_closed_form_random_sequential(oracle):
    """Random-sequential deposition without restriction: E[W^2] = t (1 - 1/L^2)."""
    L, t = 32, 5
    w2 = []
    for seed in range(40):
        h = workloads.flat(L)
        log = oracle.rs_run(h, L, INT32_MAX, rs_seed=seed + 1, t0=0, n=t)
        assert int(log[-1, 1]) == t * L * L
        w2.append(oracle.width2(L, log[-1, 1], log[-1, 2]))
    w2 = np.asarray(w2)
    expect = t * (1 - 1 / (L * L))
    se = w2.std(ddof=1) / np.sqrt(len(w2))
    assert abs(w2.mean() - expect) < 4 * se


def test_width_formula_small_cases(oracle):
    """Eq. (2) on hand-computed lattices."""
    assert oracle.width2(2, 0, 0) == 0.0
    # heights (0, 1, 0, 1): mean 1/2, mean square 1/2, W^2 = 1/4
    assert oracle.width2(2, 2, 2) == 0.25
    # heights (0, 0, 0, 3): mean 3/4, mean square 9/4, W^2 = 9/4 - 9/16 = 27/16
    assert oracle.width2(2, 3, 9) == 27 / 16
