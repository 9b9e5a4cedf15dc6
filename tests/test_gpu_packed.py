"""GPU parity of the 16-bit storage mode (RSOS_FLAG_PACKED16) against the
CPU oracle, bit for bit.

The heights live on the device as residues mod 2^16; the cases cover every
tile size D, both staging widths (uint8 with its range check and the int16
fallback), residues that wrap past a multiple of 2^16, the largest spread the
mode admits (a cone over the whole torus with N L = 24576), resume from a
checkpoint, batches, hipGraph replay, the device readout, and the full
16384^2 surface in the launch configuration the benchmark times.
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[packed] {msg}", flush=True)
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
    # L, N, D, seed, sweeps, start
    (256, 1, 8, 7, 40, "flat"),         # 16x8 tile blocks
    (512, 1, 8, 41, 30, "flat"),        # 32x8 tile blocks
    (384, 2, 8, 11, 20, "rough"),       # T = 48
    (1024, 12, 8, 43, 12, "rough"),     # N D = 96: the widest uint8 margin
    (256, 1, 4, 19, 16, "flat"),
    (256, 3, 16, 23, 8, "rough"),
    (256, 1, 2, 29, 10, "flat"),
    (2048, 1, 8, 37, 70, "flat"),       # 70 sweeps: two hipGraph replays
    (768, 2, 8, 47, 20, "high"),        # heights straddle 3 * 2^16
    (256, 1, 8, 53, 20, "top"),         # heights near 170 * 2^16 (near the S2 limit at L = 256)
    (256, 2, 32, 59, 6, "rough"),       # D = 32: 2x2 tile blocks
]


@pytest.mark.parametrize("L,N,D,seed,sweeps,start", CASES)
def test_packed_surface_matches_oracle(rsos, oracle, L, N, D, seed, sweeps, start):
    _say(f"packed surface L={L} N={N} D={D} seed={seed} sweeps={sweeps} start={start}")
    if start == "flat":
        h0 = workloads.flat(L)
    elif start == "rough":
        h0 = workloads.rough(L, N, seed=seed)
    elif start == "high":
        h0 = workloads.rough(L, N, seed=seed, base=3 * 65536 - 3 * N)
    else:
        h0 = workloads.rough(L, N, seed=seed, base=170 * 65536 - 2 * N)
    s = rsos.Surface(L, N=N, seed=seed, D=D, h0=None if start == "flat" else h0, packed=True)
    assert s.kernel_name().startswith("block_sweep16<")
    s.sweep(sweeps)
    g_log = s.log(1, sweeps)
    g_h = s.heights()
    r_h, r_log = _oracle_run(oracle, h0, L, N, D, seed, 0, sweeps)
    _compare(g_log, r_log, g_h, r_h, L)
    assert np.array_equal(s.heights_tensor().cpu().numpy(), r_h)
    s.close()


@pytest.mark.parametrize("L,N,height", [(2048, 12, 12 * 2048), (1024, 2, 900), (512, 4, 2000)])
def test_packed_cone(rsos, oracle, L, N, height):
    """Cones: steep blocks take the int16 fallback, flat ones the uint8
    staging.  The first case spans the whole torus (spread N L = 24576), so
    block references sit far from the mean on both sides."""
    _say(f"packed cone L={L} N={N} height={height}")
    h0 = workloads.cone(L, N, height, seed=L + N)
    s = rsos.Surface(L, N=N, seed=99, D=8, h0=h0, packed=True)
    s.sweep(5)
    r_h, r_log = _oracle_run(oracle, h0, L, N, 8, 99, 0, 5)
    _compare(s.log(1, 5), r_log, s.heights(), r_h, L)
    s.close()


def test_packed_resume_from_checkpoint(rsos, oracle):
    L, N, D, seed = 512, 2, 8, 202
    _say("packed resume from t0=37")
    h0 = workloads.rough(L, N, seed=3, base=70000)
    mid, _ = _oracle_run(oracle, h0, L, N, D, seed, 0, 37)
    s = rsos.Surface(L, N=N, seed=seed, D=D, h0=mid, t0=37, packed=True)
    s.sweep(9)
    r_h, r_log = _oracle_run(oracle, mid, L, N, D, seed, 37, 9)
    _compare(s.log(38, 9), r_log, s.heights(), r_h, L)


def test_packed_batch_matches_solo_oracle(rsos, oracle):
    specs = [(256, 1, 5), (512, 2, 6), (256, 4, 7), (1024, 1, 8), (384, 1, 9)]
    counts = [12, 7, 12, 3, 9]
    _say(f"packed batch {specs} counts={counts}")
    b = rsos.Batch(specs, D=8, packed=True)
    b.sweep(counts)
    for i, ((L, N, seed), n) in enumerate(zip(specs, counts)):
        r_h, r_log = _oracle_run(oracle, workloads.flat(L), L, N, 8, seed, 0, n)
        _compare(b.log(i, 1, n), r_log, b.heights(i), r_h, L)


def test_packed_invalid(rsos):
    from paper_1605_02620_amd._lib import RsosError, E_INVAL
    _say("packed invalid arguments")
    for (L, N, D) in [(16384, 2, 8), (128, 1, 8), (1024, 13, 8)]:
        with pytest.raises(RsosError) as e:
            rsos.Surface(L, N=N, D=D, packed=True)
        assert e.value.status == E_INVAL


def test_packed_full_size_first_sweeps(rsos, oracle):
    """The 16384^2 surface with 16-bit storage: the first three sweeps from
    the flat start against the oracle, every site and every sum."""
    cfg = workloads.cfg_single()
    L, N, D, seed, n = cfg.L, cfg.N, cfg.D, cfg.seed, 3
    _say(f"packed full size L={L} first {n} sweeps")
    s = rsos.Surface(L, N=N, seed=seed, D=D, packed=True)
    s.sweep(n)
    g_log = s.log(1, n)
    g_h = s.heights()
    s.close()
    r_h, r_log = _oracle_run(oracle, workloads.flat(L), L, N, D, seed, 0, n)
    _compare(g_log, r_log, g_h, r_h, L)


def test_packed_full_size_invariants(rsos):
    """2000 sweeps of the 16384^2 surface with 16-bit storage: restriction
    on every bond, S1 equal to the accepted ledger and to the heights, S2
    equal to the sum of squared heights."""
    cfg = workloads.cfg_single()
    L, N = cfg.L, cfg.N
    _say(f"packed full size invariants L={L} sweeps={cfg.sweeps}")
    s = rsos.Surface(L, N=N, seed=cfg.seed, D=cfg.D, packed=True)
    s.sweep(cfg.sweeps)
    lg = s.log(1, cfg.sweeps)
    h = s.heights().reshape(L, L).astype(np.int64)
    assert np.abs(h - np.roll(h, 1, axis=0)).max() <= N
    assert np.abs(h - np.roll(h, 1, axis=1)).max() <= N
    assert int(lg["s1"][-1]) == int(lg["accepted"].sum()) == int(h.sum())
    assert int(lg["s2"][-1]) == int((h * h).sum())
    assert np.all(np.diff(lg["s1"]) == lg["accepted"][1:])
