"""Pins of the oracle's multisurface lock-step schedule (Sec. II: many
realizations share the sequence of selected sites; each applies a selection
only with probability 1/2, its own coin).

Checked against an independent pure-Python application along injected
choices, the exact one-sweep state distribution of one realization on a
4 x 4 torus, the random-number layout re-derived from rocRAND's Philox words
(sites as for the checkerboard, coins at phase codes 8 + 2r + p), the
unrestricted closed form, and the growth exponent against the checkerboard.
"""
from collections import Counter

import numpy as np
import pytest
from scipy.stats import chi2 as chi2_dist

import workloads
from oracle import brute


@pytest.mark.parametrize("L,D,N,sweeps,start", [
    (4, 2, 1, 3, "flat"), (8, 2, 1, 4, "rough"), (8, 4, 2, 3, "rough"),
    (16, 8, 1, 3, "flat"), (32, 8, 1, 2, "rough"), (32, 16, 3, 2, "rough"),
])
def test_ms_injected_matches_python_rule(oracle, L, D, N, sweeps, start):
    rng = np.random.default_rng(L * 100 + D * 10 + N + 9)
    h0 = workloads.flat(L) if start == "flat" else workloads.rough(L, N, seed=L + D)
    origins = rng.integers(0, 2 * D, size=(sweeps, 2)).astype(np.int32)
    sites = rng.integers(0, D * D, size=sweeps * 2 * L * L).astype(np.int32)
    coins = rng.integers(0, 2, size=sweeps * 2 * L * L).astype(np.int32)
    h = h0.copy()
    log = oracle.run_ms_injected(h, L, N, D, origins, sites, coins)
    st, acc = brute.ms_apply_choices(h0, L, N, D, [tuple(o) for o in origins], sites, coins)
    assert tuple(int(v) for v in h) == st
    assert [int(a) for a in log[:, 3]] == acc


@pytest.mark.parametrize("start", ["flat", "rough"])
def test_ms_L4_D2_distribution(oracle, start):
    L, D, N = 4, 2, 1
    h0 = workloads.flat(L) if start == "flat" else workloads.rough(L, N, seed=7)
    exact = brute.ms_distribution(h0, L, N, D, 1)
    assert abs(sum(exact.values()) - 1.0) < 1e-9
    counts = Counter()
    for seed in range(120000):
        h = h0.copy().reshape(1, -1)
        oracle.run_ms(h, L, N, D, seed=seed, t0=0, n=1, log=False)
        counts[tuple(int(v) for v in h[0])] += 1
    stat, dof, unknown = brute.chi2_against(exact, counts)
    assert unknown == 0
    assert dof > 500
    assert chi2_dist.sf(stat, dof) > 1e-4, (stat, dof)


def test_ms_layout_from_rocrand_words(oracle, rocrand_philox):
    """Realization r of a seeded sweep equals the injected path fed with the
    documented layout: origin from (0, 0, s, 2); selection a of tile t in
    phase p: site field a of the words at (j, t, s, p); coin bit a mod 32 of
    word (a div 32) mod 4 at (a div 128, t, s, 8 + 2r + p)."""
    for (L, D, N, seed, s, R) in [(16, 2, 1, 21, 0, 3), (32, 8, 1, 2 ** 40 + 5, 9, 4)]:
        key = [seed & 0xFFFFFFFF, seed >> 32]
        T = L // D
        nf = len(oracle.word_fields(D, 0))
        r0 = rocrand_philox([0, 0, s, 2], key)
        origin = (int(r0[0]) % (2 * D), int(r0[1]) % (2 * D))
        h0 = np.stack([workloads.rough(L, N, seed=L + k) for k in range(R)])
        hs = h0.copy()
        oracle.run_ms(hs, L, N, D, seed=seed, t0=s, n=1)
        for r in range(R):
            sites, coins = [], []
            for p in (0, 1):
                for tid in range(T * T):
                    if (tid % T + tid // T) % 2 != p:
                        continue
                    words, cw = {}, {}
                    for a in range(2 * D * D):
                        j = a // (4 * nf)
                        if j not in words:
                            words[j] = rocrand_philox([j, tid, s, p], key)
                        sites.append(oracle.word_fields(D, int(words[j][(a % (4 * nf)) // nf]))[a % nf])
                        c = a // 128
                        if c not in cw:
                            cw[c] = rocrand_philox([c, tid, s, 8 + 2 * r + p], key)
                        coins.append((int(cw[c][(a // 32) % 4]) >> (a % 32)) & 1)
            b = h0[r].copy()
            oracle.run_ms_injected(b, L, N, D, np.array([origin], dtype=np.int32),
                                   np.array(sites, dtype=np.int32), np.array(coins, dtype=np.int32))
            assert np.array_equal(hs[r], b), r


def test_ms_unrestricted_closed_form(oracle):
    """Without the restriction each site gets Binomial(2 D^2, 1/(2 D^2))
    deposits per sweep and the total is Binomial(2 L^2, 1/2), so
    E[S1] = t L^2 and E[W^2] = t (1 - 1/(2 D^2) - 1/(2 L^2))."""
    L, D, t = 32, 4, 6
    vals, s1 = [], []
    h = np.zeros((300, L * L), dtype=np.int32)
    lg = oracle.run_ms(h, L, 2 ** 31 - 1, D, seed=77, t0=0, n=t)
    for r in range(300):
        s1.append(int(lg[r, -1, 1]))
        vals.append(oracle.width2(L, lg[r, -1, 1], lg[r, -1, 2]))
    want = t * (1 - 1 / (2 * D * D) - 1 / (2 * L * L))
    se = np.std(vals) / np.sqrt(len(vals))
    assert abs(np.mean(vals) - want) < 4 * se, (np.mean(vals), want, se)
    se1 = np.std(s1) / np.sqrt(len(s1))
    assert abs(np.mean(s1) - t * L * L) < 4 * se1


def test_ms_growth_exponent_matches_checkerboard(oracle):
    oracle.set_threads(8)
    try:
        L = 512
        h = workloads.flat(L)
        lg = oracle.run(h, L, 1, 8, seed=4, t0=0, n=256)
        hm = np.zeros((4, L * L), dtype=np.int32)
        lgm = oracle.run_ms(hm, L, 1, 8, seed=4, t0=0, n=256)
    finally:
        oracle.set_threads(0)
    ts = lg[:, 0].astype(float)
    m = (ts >= 32) & (ts <= 256)

    def beta(log):
        w2 = np.array([oracle.width2(L, a, b) for a, b in zip(log[:, 1], log[:, 2])])
        return np.polyfit(np.log(ts[m]), np.log(w2[m]), 1)[0] / 2
    b_tc = beta(lg)
    b_ms = np.mean([beta(lgm[r]) for r in range(4)])
    assert 0.21 <= b_ms <= 0.27, b_ms
    assert abs(b_ms - b_tc) < 0.02, (b_ms, b_tc)
