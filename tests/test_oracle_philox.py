"""Pins of the oracle's random-number layer.

The paper names no generator (Sec. II only says that RNG states compete with
the lattice for GPU memory); the build fixes Philox4x32-10 (Salmon et al.,
SC'11).  The oracle's implementation is pinned to rocRAND's independent
implementation of the same generator, and the bit-field split that turns a
word into in-tile sites is pinned to a worked-by-hand example.
"""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "field_extraction.txt")


def _golden_fields():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        parts = line.split()
        rows.append((int(parts[0]), int(parts[1], 16), [int(x) for x in parts[2:]]))
    return rows


def test_philox_matches_rocrand(oracle, rocrand_philox):
    rng = np.random.default_rng(1605)
    cases = [([0, 0, 0, 0], [0, 0]),
             ([0xFFFFFFFF, 0x3FFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF], [0xFFFFFFFF, 0xFFFFFFFF]),
             ([1, 2, 3, 4], [5, 6])]
    for _ in range(500):
        c = [int(v) for v in rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)]
        c[1] &= 0x3FFFFFFF  # the probe addresses the block index through a 64-bit offset
        k = [int(v) for v in rng.integers(0, 2 ** 32, size=2, dtype=np.uint64)]
        cases.append((c, k))
    for c, k in cases:
        assert list(oracle.philox(c, k)) == list(rocrand_philox(c, k)), (c, k)


@pytest.mark.parametrize("D,word,fields", _golden_fields())
def test_field_extraction_golden(oracle, D, word, fields):
    assert oracle.word_fields(D, word) == fields


def test_tile_sites_follow_documented_layout(oracle, rocrand_philox):
    """Attempt a of a tile uses call a // 4f at counter (j, tile_id, s, p),
    word (a mod 4f) // f and field a mod f; the field r gives (r mod D, r // D)."""
    seed = 0x0123456789ABCDEF
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for D in (2, 4, 8, 16, 32):
        f = oracle.word_fields(D, 0)
        nf = len(f)
        for (s, p, tid) in [(0, 0, 0), (7, 1, 12345), (2 ** 32 - 1, 0, 2 ** 20 + 3)]:
            u, v = oracle.tile_sites(D, seed, s, p, tid)
            words = {}
            for a in range(D * D):
                j = a // (4 * nf)
                if j not in words:
                    words[j] = rocrand_philox([j, tid, s, p], key)
                r = oracle.word_fields(D, int(words[j][(a % (4 * nf)) // nf]))[a % nf]
                assert (u[a], v[a]) == (r % D, r // D)


def test_origin_uses_tag_two(oracle, rocrand_philox):
    for D in (2, 8, 16):
        for seed in (0, 1, 2 ** 64 - 1):
            key = [seed & 0xFFFFFFFF, seed >> 32]
            for s in (0, 1, 999, 2 ** 32 - 1):
                r = rocrand_philox([0, 0, s, 2], key)
                assert oracle.origin(D, seed, s) == (int(r[0]) % (2 * D), int(r[1]) % (2 * D))


def test_sites_are_uniform(oracle):
    """Every in-tile site is equally likely: chi-square over many tiles."""
    from scipy.stats import chisquare
    for D in (2, 4, 8):
        counts = np.zeros(D * D)
        for tid in range(4000 // D):
            u, v = oracle.tile_sites(D, 42, 3, tid & 1, tid)
            np.add.at(counts, v * D + u, 1)
        assert chisquare(counts).pvalue > 1e-4
