"""GPU parity: librsos.so against the CPU oracle, bit for bit.

Every case compares, sweep by sweep, the exact sums (S1, S2, A) of Eq. (2)
and the final heights of the HIP path with the oracle on the same seeded
inputs.  Sizes span several tile blocks with ragged block counts, every tile
size D, both the LDS-resident path and the block path, hipGraph replay,
resume from a checkpoint produced by the oracle, and the full 16384^2
surface (its first sweeps bit for bit, and invariants after 2000 sweeps).
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[parity] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rsos():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1605_02620_amd as pkg
    return pkg


def _oracle_run(oracle, h0, L, N, D, seed, t0, n, threads=16):
    oracle.set_threads(threads)
    try:
        h = h0.copy()
        lg = oracle.run(h, L, N, D, seed=seed, t0=t0, n=n)
    finally:
        oracle.set_threads(0)
    return h, lg


def _compare(gpu_log, ref_log, gpu_h, ref_h, L):
    assert np.array_equal(gpu_log["t"], ref_log[:, 0])
    for k, name in ((1, "s1"), (2, "s2"), (3, "accepted")):
        bad = np.nonzero(gpu_log[name] != ref_log[:, k])[0]
        assert bad.size == 0, f"{name} differs first at t={int(ref_log[bad[0], 0])}"
    diff = np.nonzero(gpu_h != ref_h)[0]
    assert diff.size == 0, f"heights differ at {diff.size} sites, first (x={diff[0] % L}, y={diff[0] // L})"


CASES = [
    # L, N, D, seed, sweeps, start   (path: LDS for L <= 128, block otherwise)
    (64, 1, 8, 1, 1024, "flat"),       # the small configuration, whole run
    (32, 2, 4, 3, 200, "rough"),
    (128, 1, 16, 5, 100, "flat"),
    (256, 1, 8, 7, 40, "flat"),        # block path, 16x8 tile blocks
    (384, 2, 8, 11, 20, "rough"),      # T = 48: ragged vs powers of two
    (272, 1, 8, 13, 12, "flat"),       # T = 34: only 2x2 tile blocks fit
    (512, 4, 8, 17, 16, "rough"),
    (256, 1, 4, 19, 16, "flat"),
    (256, 3, 16, 23, 8, "rough"),
    (256, 1, 2, 29, 10, "flat"),
    (256, 2 ** 31 - 1, 8, 31, 6, "flat"),  # no restriction: every attempt accepted
    (2048, 1, 8, 37, 60, "flat"),      # 256 blocks per sweep
    (64, 1, 32, 41, 40, "flat"),       # D = 32: LDS path
    (256, 2, 32, 43, 6, "rough"),      # D = 32: 2x2 tile blocks, int8 staging
    (192, 5, 32, 47, 4, "rough"),      # D = 32, N D = 160: int32 staging
]


@pytest.mark.parametrize("L,N,D,seed,sweeps,start", CASES)
def test_surface_matches_oracle(rsos, oracle, L, N, D, seed, sweeps, start):
    _say(f"surface L={L} N={N} D={D} seed={seed} sweeps={sweeps} start={start}")
    h0 = workloads.flat(L) if start == "flat" else workloads.rough(L, min(N, 4), seed=seed)
    s = rsos.Surface(L, N=N, seed=seed, D=D, h0=None if start == "flat" else h0)
    s.sweep(sweeps)
    g_log = s.log(1, sweeps)
    g_h = s.heights()
    r_h, r_log = _oracle_run(oracle, h0, L, N, D, seed, 0, sweeps)
    _compare(g_log, r_log, g_h, r_h, L)
    w = s.width()
    assert w["t"] == sweeps and w["w2"] == oracle.width2(L, r_log[-1, 1], r_log[-1, 2])
    s.close()


@pytest.mark.parametrize("L,N,height", [(1024, 2, 900), (2048, 1, 700), (512, 4, 2000)])
def test_mixed_staging_widths(rsos, oracle, L, N, height):
    """A cone: blocks near the apex exceed the narrow LDS staging and are
    re-run with wider staging, flat blocks are not; both agree with the
    oracle bit for bit, over sweeps that move the cone's slopes."""
    _say(f"cone L={L} N={N} height={height}")
    h0 = workloads.cone(L, N, height, seed=L + N)
    s = rsos.Surface(L, N=N, seed=99, D=8, h0=h0)
    s.sweep(6)
    r_h, r_log = _oracle_run(oracle, h0, L, N, 8, 99, 0, 6)
    _compare(s.log(1, 6), r_log, s.heights(), r_h, L)
    s.close()


def test_graph_replay_and_split_calls(rsos, oracle):
    """Sweeps issued as one long call on a side stream (hipGraph replays of
    32 sweeps), as many short calls, and as a mix give the same bits."""
    import torch
    L, N, D, seed, n = 256, 1, 8, 101, 100
    _say(f"graph replay L={L} sweeps={n}")
    st = torch.cuda.Stream()
    a = rsos.Surface(L, N=N, seed=seed, D=D, stream=st)
    a.sweep(n)
    b = rsos.Surface(L, N=N, seed=seed, D=D)
    for k in (1, 2, 3, 30, 64):
        b.sweep(k)
    assert a.time() == b.time() == n
    assert np.array_equal(a.heights(), b.heights())
    assert np.array_equal(a.log(1, n), b.log(1, n))
    r_h, r_log = _oracle_run(oracle, workloads.flat(L), L, N, D, seed, 0, n)
    _compare(a.log(1, n), r_log, a.heights(), r_h, L)


def test_timing_mode(rsos, oracle):
    """The timing mode (each sweep's kernels bracketed by events the runtime
    records at their start and end) reports one duration per sweep and
    changes no bit of the result; packed storage and a batch as well."""
    import torch
    L, N, D, seed, n = 512, 1, 8, 31, 12
    _say(f"timing mode L={L} sweeps={n}")
    for packed in (False, True):
        st = torch.cuda.Stream()
        a = rsos.Surface(L, N=N, seed=seed, D=D, stream=st, packed=packed)
        a.sweep(4)
        a.timing(True)
        a.sweep(n - 4)
        launches, mean_ms, total_ms = a.timing_read()
        a.timing(False)
        assert launches == n - 4 and 0 < mean_ms and abs(total_ms - mean_ms * launches) < 1e-6 * total_ms + 1e-9
        r_h, r_log = _oracle_run(oracle, workloads.flat(L), L, N, D, seed, 0, n)
        _compare(a.log(1, n), r_log, a.heights(), r_h, L)
        a.close()


def test_resume_from_checkpoint(rsos, oracle):
    L, N, D, seed = 256, 2, 8, 202
    _say("resume from t0=37")
    h0 = workloads.rough(L, N, seed=3)
    mid, _ = _oracle_run(oracle, h0, L, N, D, seed, 0, 37)
    s = rsos.Surface(L, N=N, seed=seed, D=D, h0=mid, t0=37)
    s.sweep(9)
    r_h, r_log = _oracle_run(oracle, mid, L, N, D, seed, 37, 9)
    _compare(s.log(38, 9), r_log, s.heights(), r_h, L)
    rec = s.log(37, 1)[0]
    assert (rec["s1"], rec["s2"], rec["accepted"]) == (int(mid.astype(np.int64).sum()),
                                                        int((mid.astype(np.int64) ** 2).sum()), 0)


def test_batch_matches_solo_oracle(rsos, oracle):
    specs = [(256, 1, 5), (512, 2, 6), (256, 4, 7), (1024, 1, 8), (384, 1, 9)]
    counts = [12, 7, 12, 3, 9]
    _say(f"batch {specs} counts={counts}")
    b = rsos.Batch(specs, D=8)
    b.sweep(counts)
    ws = b.width()
    for i, ((L, N, seed), n) in enumerate(zip(specs, counts)):
        r_h, r_log = _oracle_run(oracle, workloads.flat(L), L, N, 8, seed, 0, n)
        _compare(b.log(i, 1, n), r_log, b.heights(i), r_h, L)
        assert ws[i]["t"] == n
    b.sweep(2)  # everyone advances two more
    for i, ((L, N, seed), n) in enumerate(zip(specs, counts)):
        assert b.width()[i]["t"] == n + 2


def test_empty_work(rsos, oracle):
    """Zero-sweep calls change nothing (single surface, and surfaces given 0
    sweeps inside a batch next to surfaces that advance, on both the tile-
    block and the LDS paths); the work that follows is still bit-exact."""
    _say("empty work")
    L, N, seed = 256, 1, 61
    s = rsos.Surface(L, N=N, seed=seed, D=8)
    s.sweep(0).sweep(0)
    w = s.width()
    assert (w["t"], w["s1"], w["s2"], w["accepted"]) == (0, 0, 0, 0)
    assert not s.heights().any()
    s.sweep(3).sweep(0)
    r_h, r_log = _oracle_run(oracle, workloads.flat(L), L, N, 8, seed, 0, 3)
    _compare(s.log(1, 3), r_log, s.heights(), r_h, L)
    s.close()
    specs = [(256, 1, 62), (64, 1, 63), (512, 2, 64), (128, 1, 65)]
    counts = [0, 5, 0, 4]
    b = rsos.Batch(specs, D=8)
    b.sweep(counts)
    ws = b.width()
    for i, ((Lb, Nb, sb), n) in enumerate(zip(specs, counts)):
        assert ws[i]["t"] == n
        if n == 0:
            assert not b.heights(i).any() and ws[i]["s1"] == 0
        else:
            r_h, r_log = _oracle_run(oracle, workloads.flat(Lb), Lb, Nb, 8, sb, 0, n)
            _compare(b.log(i, 1, n), r_log, b.heights(i), r_h, Lb)
    b.sweep([0, 0, 0, 0])
    assert [int(x) for x in b.width()["t"]] == counts
    b.close()


def test_invalid_arguments(rsos):
    from paper_1605_02620_amd._lib import RsosError, E_INVAL, E_RSOS
    _say("invalid arguments")
    with pytest.raises(RsosError) as e:
        rsos.Surface(24, N=1, D=8)
    assert e.value.status == E_INVAL
    with pytest.raises(RsosError) as e:
        rsos.Surface(64, N=1, D=8, h0=workloads.violating(64, 1, seed=2))
    assert e.value.status == E_RSOS
    with pytest.raises(RsosError) as e:
        rsos.Surface(64, N=0, D=8)
    assert e.value.status == E_INVAL


def test_full_size_first_sweeps(rsos, oracle):
    """The 16384^2 surface in the launch configuration the benchmark times:
    both sides run the first three sweeps from the flat start; every site
    and every sum must agree."""
    cfg = workloads.cfg_single()
    L, N, D, seed, n = cfg.L, cfg.N, cfg.D, cfg.seed, 3
    _say(f"full size L={L} first {n} sweeps")
    s = rsos.Surface(L, N=N, seed=seed, D=D)
    s.sweep(n)
    g_log = s.log(1, n)
    g_h = s.heights()
    s.close()
    r_h, r_log = _oracle_run(oracle, workloads.flat(L), L, N, D, seed, 0, n)
    _compare(g_log, r_log, g_h, r_h, L)


def test_max_size_first_sweeps(rsos, oracle):
    """The largest lattice the library accepts, L = 65536 (2^32 sites, 16 GiB
    per int32 buffer; every site index needs 64 bits on both sides): the
    first sweep from the flat start, every site and every sum."""
    L, N, D, seed, n = 65536, 1, 8, 21, 1
    _say(f"maximum size L={L} first {n} sweeps")
    s = rsos.Surface(L, N=N, seed=seed, D=D, log_cap=8)
    s.sweep(n)
    g_log = s.log(1, n)
    g_h = s.heights()
    s.close()
    del s
    _say("maximum size: oracle")
    h = workloads.flat(L)
    oracle.set_threads(16)
    try:
        r_log = oracle.run(h, L, N, D, seed=seed, t0=0, n=n)
    finally:
        oracle.set_threads(0)
    _compare(g_log, r_log, g_h, h, L)


def test_full_size_invariants(rsos):
    """2000 sweeps of the 16384^2 surface: the restriction holds everywhere,
    S1 equals the accepted-deposit ledger, and S2 matches the heights."""
    cfg = workloads.cfg_single()
    L, N = cfg.L, cfg.N
    _say(f"full size invariants L={L} sweeps={cfg.sweeps}")
    s = rsos.Surface(L, N=N, seed=cfg.seed, D=cfg.D)
    s.sweep(cfg.sweeps)
    lg = s.log(1, cfg.sweeps)
    h = s.heights().reshape(L, L).astype(np.int64)
    assert np.abs(h - np.roll(h, 1, axis=0)).max() <= N
    assert np.abs(h - np.roll(h, 1, axis=1)).max() <= N
    assert int(lg["s1"][-1]) == int(lg["accepted"].sum()) == int(h.sum())
    assert int(lg["s2"][-1]) == int((h * h).sum())
    assert np.all(np.diff(lg["s1"]) == lg["accepted"][1:])
    w = s.width()
    assert 0 < w["w2"] < 100
