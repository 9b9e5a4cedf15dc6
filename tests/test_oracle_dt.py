"""Pins of the oracle's double-tiling schedule (Sec. II: tiles split into
2 x 2 sub-tiles, 4 sets of sub-tiles updated in turn).

Checked against an independent pure-Python application of the rule along
injected choices, the exact state distribution after one sweep of a 4 x 4
torus, the random-number layout re-derived from rocRAND's Philox words
(phase codes 4..7), the unrestricted closed form, and the growth exponent
against the checkerboard schedule (Sec. III.C: the decomposition must not
change the exponents).
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
def test_dt_injected_matches_python_rule(oracle, L, D, N, sweeps, start):
    rng = np.random.default_rng(L * 100 + D * 10 + N + 5)
    h0 = workloads.flat(L) if start == "flat" else workloads.rough(L, N, seed=L + D)
    origins = rng.integers(0, 2 * D, size=(sweeps, 2)).astype(np.int32)
    sites = rng.integers(0, D * D, size=sweeps * L * L).astype(np.int32)
    h = h0.copy()
    log = oracle.run_dt_injected(h, L, N, D, origins, sites)
    st, acc = brute.dt_apply_choices(h0, L, N, D, [tuple(o) for o in origins], sites)
    assert tuple(int(v) for v in h) == st
    assert [int(a) for a in log[:, 3]] == acc


@pytest.mark.parametrize("start", ["flat", "rough"])
def test_dt_L4_D2_distribution(oracle, start):
    """One double-tiling sweep on a 4 x 4 torus with 2 x 2 sub-tiles: 16
    origins, one sub-tile per set, 4 attempts each."""
    L, D, N = 4, 2, 1
    h0 = workloads.flat(L) if start == "flat" else workloads.rough(L, N, seed=7)
    exact = brute.dt_distribution(h0, L, N, D, 1)
    assert abs(sum(exact.values()) - 1.0) < 1e-9
    counts = Counter()
    for seed in range(120000):
        h = h0.copy()
        oracle.run_dt(h, L, N, D, seed=seed, t0=0, n=1, log=False)
        counts[tuple(int(v) for v in h)] += 1
    stat, dof, unknown = brute.chi2_against(exact, counts)
    assert unknown == 0
    assert dof > 500
    assert chi2_dist.sf(stat, dof) > 1e-4, (stat, dof)


def test_dt_layout_from_rocrand_words(oracle, rocrand_philox):
    """A seeded double-tiling sweep equals the injected path fed with the
    origin from counter (0, 0, s, 2) and, for set k, the fields of the words
    at counters (j, sub_id, s, 4 + k) in the documented layout."""
    for (L, D, N, seed, s) in [(16, 2, 1, 11, 0), (32, 4, 2, 12, 5), (32, 8, 1, 2 ** 40 + 3, 77)]:
        key = [seed & 0xFFFFFFFF, seed >> 32]
        T = L // D
        nf = len(oracle.word_fields(D, 0))
        r = rocrand_philox([0, 0, s, 2], key)
        origin = (int(r[0]) % (2 * D), int(r[1]) % (2 * D))
        sites = []
        for k in range(4):
            for sid in range(T * T):
                if (sid % T) % 2 + 2 * ((sid // T) % 2) != k:
                    continue
                words = {}
                for a in range(D * D):
                    j = a // (4 * nf)
                    if j not in words:
                        words[j] = rocrand_philox([j, sid, s, 4 + k], key)
                    sites.append(oracle.word_fields(D, int(words[j][(a % (4 * nf)) // nf]))[a % nf])
        h0 = workloads.rough(L, N, seed=L + N)
        a = h0.copy()
        oracle.run_dt(a, L, N, D, seed=seed, t0=s, n=1)
        b = h0.copy()
        oracle.run_dt_injected(b, L, N, D, np.array([origin], dtype=np.int32), np.array(sites, dtype=np.int32))
        assert np.array_equal(a, b)


def test_dt_unrestricted_closed_form(oracle):
    """Without the restriction every attempt is accepted: S1 = t L^2, and
    each site gets Binomial(D^2, 1/D^2) deposits per sweep, so
    E[W^2] = t (1 - 1/D^2)."""
    L, D, t = 32, 4, 6
    vals = []
    for seed in range(300):
        h = workloads.flat(L)
        lg = oracle.run_dt(h, L, 2 ** 31 - 1, D, seed=seed, t0=0, n=t)
        assert int(lg[-1, 1]) == t * L * L
        vals.append(oracle.width2(L, lg[-1, 1], lg[-1, 2]))
    want = float(brute.tiled_rd_w2_mean(t, D))
    se = np.std(vals) / np.sqrt(len(vals))
    assert abs(np.mean(vals) - want) < 4 * se, (np.mean(vals), want, se)


def test_dt_growth_exponent_matches_checkerboard(oracle):
    oracle.set_threads(8)
    try:
        L = 512
        ws = {}
        for name, fn in (("tc", oracle.run), ("dt", oracle.run_dt)):
            h = workloads.flat(L)
            lg = fn(h, L, 1, 8, seed=4, t0=0, n=256)
            ts = lg[:, 0].astype(float)
            w2 = np.array([oracle.width2(L, a, b) for a, b in zip(lg[:, 1], lg[:, 2])])
            m = (ts >= 32) & (ts <= 256)
            ws[name] = np.polyfit(np.log(ts[m]), np.log(w2[m]), 1)[0] / 2
    finally:
        oracle.set_threads(0)
    assert 0.21 <= ws["dt"] <= 0.27, ws
    assert abs(ws["dt"] - ws["tc"]) < 0.02, ws
