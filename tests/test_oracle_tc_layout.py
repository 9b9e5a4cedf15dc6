"""Pin of how the oracle's seeded tile-checkerboard sweep composes its random
streams (Sec. II: domain decomposition whose origin moves randomly after
each sweep; independent domains of one set updated by independent workers).

The per-tile stream and the field split have pins of their own; this one
fixes which stream each tile receives and in which phase.  The choices are
rebuilt here from rocRAND's own Philox4x32-10 words in the documented
layout, with no oracle code:
  origin of sweep s   = words 0, 1 of counter (0, 0, s, 2), each mod 2D;
  phase p, tile (tx, ty) of the shifted frame with (tx + ty) mod 2 = p,
  tile_id = ty (L/D) + tx   -> attempt a takes field a mod f of word
  (a mod 4f) div f of counter (a div 4f, tile_id, s, p), f = floor(32/b),
  b = 2 log2 D bits, lowest field first.
A seeded oracle sweep must equal both the oracle's injected path and an
independent pure-Python application of the rule fed with those choices.
A transposed tile_id, a swapped phase code or a wrong tile <-> site mapping
in the seeded path changes the result.
"""
import numpy as np
import pytest

import workloads
from oracle import brute


def _fields(D, word):
    b = 2 * (D.bit_length() - 1)
    f = 32 // b
    return [(int(word) >> (k * b)) & (D * D - 1) for k in range(f)]


def _rocrand_choices(philox, L, D, seed, s):
    key = [seed & 0xFFFFFFFF, seed >> 32]
    T = L // D
    f = len(_fields(D, 0))
    r = philox([0, 0, s, 2], key)
    origin = (int(r[0]) % (2 * D), int(r[1]) % (2 * D))
    sites = []
    for p in (0, 1):
        for tid in range(T * T):
            tx, ty = tid % T, tid // T
            if (tx + ty) % 2 != p:
                continue
            words = {}
            for a in range(D * D):
                j = a // (4 * f)
                if j not in words:
                    words[j] = philox([j, tid, s, p], key)
                sites.append(_fields(D, words[j][(a % (4 * f)) // f])[a % f])
    return origin, sites


@pytest.mark.parametrize("L,D,N,seed,s0,sweeps", [
    (16, 2, 1, 11, 0, 2),
    (32, 4, 2, 2 ** 40 + 12, 5, 2),
    (32, 8, 1, 1, 0, 3),
    (48, 8, 3, 0xDEADBEEFCAFEF00D, 2 ** 32 - 2, 2),
    (64, 16, 2, 2 ** 63 + 7, 1000, 1),
    (64, 32, 1, 77, 2 ** 32 - 1, 1),
])
def test_tc_layout_from_rocrand_words(oracle, rocrand_philox, L, D, N, seed, s0, sweeps):
    h0 = workloads.rough(L, N, seed=L + D + N)
    seeded = h0.copy()
    lg = oracle.run(seeded, L, N, D, seed=seed, t0=s0, n=sweeps)
    origins, sites = [], []
    for s in range(s0, s0 + sweeps):
        o, st = _rocrand_choices(rocrand_philox, L, D, seed, s)
        origins.append(o)
        sites += st
    injected = h0.copy()
    lg_inj = oracle.run_injected(injected, L, N, D, np.array(origins, dtype=np.int32),
                                 np.array(sites, dtype=np.int32))
    assert np.array_equal(seeded, injected)
    assert np.array_equal(lg[:, 1:], lg_inj[:, 1:])
    st, acc = brute.tc_apply_choices(h0, L, N, D, origins, sites)
    assert tuple(int(v) for v in seeded) == st
    assert [int(a) for a in lg[:, 3]] == acc


def test_tc_layout_distinguishes_tiles_and_phases(oracle, rocrand_philox):
    """The pin has teeth: choices built with the tile_id transposed, or with
    the phase codes swapped, give a different trajectory on a rough start."""
    L, D, N, seed, s = 32, 8, 1, 5, 3
    h0 = workloads.rough(L, N, seed=9)
    a = h0.copy()
    oracle.run(a, L, N, D, seed=seed, t0=s, n=1)
    o, sites = _rocrand_choices(rocrand_philox, L, D, seed, s)
    T = L // D
    key = [seed, 0]

    def build(tile_code, phase_code):
        out = []
        f = len(_fields(D, 0))
        for p in (0, 1):
            for tid in range(T * T):
                tx, ty = tid % T, tid // T
                if (tx + ty) % 2 != p:
                    continue
                w = {}
                for k in range(D * D):
                    j = k // (4 * f)
                    if j not in w:
                        w[j] = rocrand_philox([j, tile_code(tx, ty), s, phase_code(p)], key)
                    out.append(_fields(D, w[j][(k % (4 * f)) // f])[k % f])
        return out

    assert build(lambda tx, ty: ty * T + tx, lambda p: p) == sites
    for wrong in (build(lambda tx, ty: tx * T + ty, lambda p: p), build(lambda tx, ty: ty * T + tx, lambda p: 1 - p)):
        b = h0.copy()
        oracle.run_injected(b, L, N, D, np.array([o], dtype=np.int32), np.array(wrong, dtype=np.int32))
        assert not np.array_equal(a, b)
