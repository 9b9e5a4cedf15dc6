"""Exact enumeration for tiny RSOS lattices (L <= 4).

TEST INFRASTRUCTURE ONLY.  Pure Python and numpy.  It
propagates the full probability distribution over lattice states attempt by
attempt instead of sampling paths, so the C oracle's sampled frequencies can
be chi-square tested against exact probabilities (float64 weights), and it
solves the stationary Markov chain of small random-sequential lattices in
exact rationals.

The model is the one of Kelling, Odor & Gemming, Sec. I: deposition at a
uniformly random site, accepted if afterwards every nearest-neighbour height
difference is at most N in magnitude, on an L x L periodic square lattice.
The schedule enumerated for the tiled case is the domain decomposition of
Sec. II in its tile-checkerboard reading: origin uniform over [0, 2D)^2,
colour-0 tiles then colour-1 tiles, D*D uniform in-tile attempts per tile.
"""
from __future__ import annotations

from collections import defaultdict
from fractions import Fraction
import numpy as np


def _neighbours(L, x, y):
    return [((x + 1) % L, y), ((x - 1) % L, y), (x, (y + 1) % L), (x, (y - 1) % L)]


def deposit(state, L, N, x, y):
    """The RSOS rule on a tuple state (row-major); returns the new tuple."""
    i = y * L + x
    after = state[i] + 1
    for (nx, ny) in _neighbours(L, x, y):
        if abs(after - state[ny * L + nx]) > N:
            return state
    lst = list(state)
    lst[i] = after
    return tuple(lst)


BITS = 4  # bits per site in the packed state code (heights 0..15)


def encode(state):
    code = 0
    for i, v in enumerate(state):
        assert 0 <= int(v) < (1 << BITS)
        code |= int(v) << (BITS * i)
    return code


def decode(code, n):
    m = (1 << BITS) - 1
    return tuple((int(code) >> (BITS * i)) & m for i in range(n))


def _deposit_codes(codes, L, N, x, y):
    """The RSOS rule applied to an array of packed states at one site."""
    m = np.uint64((1 << BITS) - 1)
    i = y * L + x
    hi = (codes >> np.uint64(BITS * i)) & m
    after = hi.astype(np.int64) + 1
    ok = np.ones(codes.shape, dtype=bool)
    for (nx, ny) in _neighbours(L, x, y):
        j = ny * L + nx
        nb = ((codes >> np.uint64(BITS * j)) & m).astype(np.int64)
        ok &= np.abs(after - nb) <= N
    if np.any(ok & (after >= (1 << BITS))):
        raise OverflowError("height exceeds the packed code range")
    return codes + (ok.astype(np.uint64) << np.uint64(BITS * i))


def _merge(codes, probs):
    u, inv = np.unique(codes, return_inverse=True)
    return u, np.bincount(inv.ravel(), weights=probs, minlength=u.size)


def _attempt_uniform(codes, probs, L, N, sites):
    """One attempt at a site drawn uniformly from `sites` (float64 weights)."""
    w = 1.0 / len(sites)
    nc = [_deposit_codes(codes, L, N, x, y) for (x, y) in sites]
    return _merge(np.concatenate(nc), np.tile(probs * w, len(sites)))


def rs_distribution(h0, L, N, n_attempts):
    """Exact state distribution (float64 probabilities) after n
    random-sequential attempts, as {state tuple: probability}."""
    codes = np.array([encode(h0)], dtype=np.uint64)
    probs = np.ones(1)
    sites = [(x, y) for y in range(L) for x in range(L)]
    for _ in range(n_attempts):
        codes, probs = _attempt_uniform(codes, probs, L, N, sites)
    return {decode(c, L * L): float(p) for c, p in zip(codes, probs)}


def _tc_sweep_codes(codes, probs, L, N, D):
    T = L // D
    shifts = [(ox, oy) for oy in range(2 * D) for ox in range(2 * D)]
    outc, outp = [], []
    for (ox, oy) in shifts:
        c, pr = codes, probs
        for p in (0, 1):
            for ty in range(T):
                for tx in range(T):
                    if (tx + ty) % 2 != p:
                        continue
                    cells = [((ox + tx * D + u) % L, (oy + ty * D + v) % L)
                             for v in range(D) for u in range(D)]
                    for _ in range(D * D):
                        c, pr = _attempt_uniform(c, pr, L, N, cells)
        outc.append(c)
        outp.append(pr / len(shifts))
    return _merge(np.concatenate(outc), np.concatenate(outp))


def _dt_sweep_codes(codes, probs, L, N, D):
    T = L // D
    shifts = [(ox, oy) for oy in range(2 * D) for ox in range(2 * D)]
    outc, outp = [], []
    for (ox, oy) in shifts:
        c, pr = codes, probs
        for k in range(4):
            for sy in range(T):
                for sx in range(T):
                    if (sx % 2) + 2 * (sy % 2) != k:
                        continue
                    cells = [((ox + sx * D + u) % L, (oy + sy * D + v) % L)
                             for v in range(D) for u in range(D)]
                    for _ in range(D * D):
                        c, pr = _attempt_uniform(c, pr, L, N, cells)
        outc.append(c)
        outp.append(pr / len(shifts))
    return _merge(np.concatenate(outc), np.concatenate(outp))


def dt_distribution(h0, L, N, D, n_sweeps):
    """Exact state distribution after n sweeps of the double-tiling
    schedule (4 sets of sub-tiles by their position in the 2 x 2 tile,
    updated in turn; origin uniform over [0, 2D)^2)."""
    codes = np.array([encode(h0)], dtype=np.uint64)
    probs = np.ones(1)
    for _ in range(n_sweeps):
        codes, probs = _dt_sweep_codes(codes, probs, L, N, D)
    return {decode(c, L * L): float(p) for c, p in zip(codes, probs)}


def dt_apply_choices(h0, L, N, D, origins, sites):
    """Double-tiling sweeps along injected choices, in pure Python: per
    sweep and set k, the sub-tiles with (sx mod 2) + 2 (sy mod 2) = k in
    increasing sub_id, D*D in-tile indices each."""
    T = L // D
    st = tuple(int(v) for v in h0)
    pos = 0
    acc = []
    for (ox, oy) in origins:
        a = 0
        for k in range(4):
            for sid in range(T * T):
                sx, sy = sid % T, sid // T
                if (sx % 2) + 2 * (sy % 2) != k:
                    continue
                for _ in range(D * D):
                    r = int(sites[pos]); pos += 1
                    x = (ox + sx * D + r % D) % L
                    y = (oy + sy * D + r // D) % L
                    nxt = deposit(st, L, N, x, y)
                    a += nxt != st
                    st = nxt
        acc.append(a)
    return st, acc


def _ms_sweep_codes(codes, probs, L, N, D):
    """One lock-step sweep of a single realization: per tile, 2 D^2
    selections, each applied with probability 1/2 at a uniform in-tile site."""
    T = L // D
    shifts = [(ox, oy) for oy in range(2 * D) for ox in range(2 * D)]
    outc, outp = [], []
    for (ox, oy) in shifts:
        c, pr = codes, probs
        for p in (0, 1):
            for ty in range(T):
                for tx in range(T):
                    if (tx + ty) % 2 != p:
                        continue
                    cells = [((ox + tx * D + u) % L, (oy + ty * D + v) % L)
                             for v in range(D) for u in range(D)]
                    for _ in range(2 * D * D):
                        c2, p2 = _attempt_uniform(c, pr, L, N, cells)
                        c, pr = _merge(np.concatenate([c, c2]), np.concatenate([pr * 0.5, p2 * 0.5]))
        outc.append(c)
        outp.append(pr / len(shifts))
    return _merge(np.concatenate(outc), np.concatenate(outp))


def ms_distribution(h0, L, N, D, n_sweeps):
    """Exact state distribution of one realization of the lock-step
    schedule after n sweeps (its coins make each selection a fair mixture
    of doing nothing and a uniform in-tile attempt)."""
    codes = np.array([encode(h0)], dtype=np.uint64)
    probs = np.ones(1)
    for _ in range(n_sweeps):
        codes, probs = _ms_sweep_codes(codes, probs, L, N, D)
    return {decode(c, L * L): float(p) for c, p in zip(codes, probs)}


def ms_apply_choices(h0, L, N, D, origins, sites, coins):
    """One lock-step realization along injected choices, pure Python: per
    sweep and colour, tiles in increasing tile_id, 2 D^2 (site, coin)
    pairs each."""
    T = L // D
    st = tuple(int(v) for v in h0)
    pos = 0
    acc = []
    for (ox, oy) in origins:
        a = 0
        for p in (0, 1):
            for tid in range(T * T):
                tx, ty = tid % T, tid // T
                if (tx + ty) % 2 != p:
                    continue
                for _ in range(2 * D * D):
                    r, coin = int(sites[pos]), int(coins[pos]); pos += 1
                    if not coin:
                        continue
                    x = (ox + tx * D + r % D) % L
                    y = (oy + ty * D + r // D) % L
                    nxt = deposit(st, L, N, x, y)
                    a += nxt != st
                    st = nxt
        acc.append(a)
    return st, acc


def tc_distribution(h0, L, N, D, n_sweeps):
    """Exact state distribution (float64 probabilities) after n sweeps of
    the tile-checkerboard schedule, as {state tuple: probability}."""
    codes = np.array([encode(h0)], dtype=np.uint64)
    probs = np.ones(1)
    for _ in range(n_sweeps):
        codes, probs = _tc_sweep_codes(codes, probs, L, N, D)
    return {decode(c, L * L): float(p) for c, p in zip(codes, probs)}


def width2_exact(state, L):
    """Eq. (2) as an exact rational."""
    n = L * L
    s1 = sum(state)
    s2 = sum(v * v for v in state)
    return Fraction(n * s2 - s1 * s1, n * n)


def rs_stationary_w2(L, N, exact=False):
    """Stationary <W^2> of random-sequential RSOS on an L x L torus.

    The chain on relative heights h - h(0,0) is finite (deposition at (0,0)
    lowers every relative height by one).  Its stationary law solves
    pi P = pi, sum pi = 1: in exact rationals (Gauss-Jordan) when `exact`,
    else in float64 (numpy).  Returns (number of states, <W^2>)."""
    n = L * L
    start = tuple([0] * n)
    index = {start: 0}
    states = [start]
    trans = []
    k = 0
    while k < len(states):
        st = states[k]
        row = defaultdict(int)
        for y in range(L):
            for x in range(L):
                nxt = deposit(st, L, N, x, y)
                base = nxt[0]
                rel = tuple(v - base for v in nxt)
                if rel not in index:
                    index[rel] = len(states)
                    states.append(rel)
                row[index[rel]] += 1  # in units of 1/n
        trans.append(row)
        k += 1
    m = len(states)
    if exact:
        A = [[Fraction(0)] * m for _ in range(m)]
        for i, row in enumerate(trans):
            for j, c in row.items():
                A[j][i] += Fraction(c, n)
            A[i][i] -= 1
        A[m - 1] = [Fraction(1)] * m
        b = [Fraction(0)] * m
        b[m - 1] = Fraction(1)
        pi = _solve(A, b)
        return m, sum(p * width2_exact(st, L) for p, st in zip(pi, states))
    A = np.zeros((m, m))
    for i, row in enumerate(trans):
        for j, c in row.items():
            A[j, i] += c / n
        A[i, i] -= 1.0
    A[m - 1, :] = 1.0
    b = np.zeros(m)
    b[m - 1] = 1.0
    pi = np.linalg.solve(A, b)
    return m, float(sum(p * float(width2_exact(st, L)) for p, st in zip(pi, states)))


def _solve(A, b):
    m = len(A)
    M = [row[:] + [b[i]] for i, row in enumerate(A)]
    for c in range(m):
        piv = next(r for r in range(c, m) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        inv = 1 / M[c][c]
        M[c] = [v * inv for v in M[c]]
        for r in range(m):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * bb for a, bb in zip(M[r], M[c])]
    return [M[i][m] for i in range(m)]


def chi2_against(exact, counts, min_expected=5.0):
    """Pearson chi-square of observed state counts against exact probabilities.

    States with small expected counts are pooled into one bin.  Returns
    (statistic, degrees of freedom, number of observed states absent from
    `exact`)."""
    total = sum(counts.values())
    stat = 0.0
    dof = -1
    pool_e = 0.0
    pool_o = 0
    unknown = sum(c for st, c in counts.items() if st not in exact)
    for st, pr in exact.items():
        e = float(pr) * total
        o = counts.get(st, 0)
        if e < min_expected:
            pool_e += e
            pool_o += o
            continue
        stat += (o - e) ** 2 / e
        dof += 1
    if pool_e > 0:
        stat += (pool_o - pool_e) ** 2 / pool_e
        dof += 1
    return stat, dof, unknown


def tiled_rd_w2_mean(t, D):
    """Closed form for unrestricted deposition (N large) under the tiled
    schedule: each site receives Binomial(D^2, 1/D^2) deposits per sweep and
    the mean height is exactly t, so E[W^2] = t (1 - 1/D^2)."""
    return Fraction(t) * (1 - Fraction(1, D * D))


def tc_apply_choices(h0, L, N, D, origins, sites):
    """Applies tile-checkerboard sweeps along injected choices, in pure Python:
    origins[i] = (ox, oy) of sweep i; sites lists, per sweep and phase, the
    tiles of that colour in increasing tile_id = ty*(L/D) + tx, D*D in-tile
    indices r = v*D + u each.  Returns (final state, accepted per sweep)."""
    T = L // D
    st = tuple(int(v) for v in h0)
    pos = 0
    acc = []
    for (ox, oy) in origins:
        a = 0
        for p in (0, 1):
            for tid in range(T * T):
                tx, ty = tid % T, tid // T
                if (tx + ty) % 2 != p:
                    continue
                for _ in range(D * D):
                    r = int(sites[pos]); pos += 1
                    x = (ox + tx * D + r % D) % L
                    y = (oy + ty * D + r // D) % L
                    nxt = deposit(st, L, N, x, y)
                    a += nxt != st
                    st = nxt
        acc.append(a)
    return st, acc
