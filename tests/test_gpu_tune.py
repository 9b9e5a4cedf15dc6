"""GPU tests of the autotuner: no launch configuration it can choose changes
a result.  Every candidate of several keys is forced in turn and compared
bit for bit with the CPU oracle; so are the configurations it actually
chooses, alone and in batches that run several kernel instances per sweep,
and jobs of the serving engine with tuned choices.  The paper chooses its
tile layout for its GPU (Sec. II); here only the result-neutral launch
knobs are tuned, never the domain size D."""
import os
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[tune] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rsos():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1605_02620_amd as pkg
    from paper_1605_02620_amd import surface
    surface.tune_clear()
    yield pkg
    surface.tune_clear()


def _oracle(oracle, h0, L, N, D, seed, n, schedule="checkerboard"):
    oracle.set_threads(16)
    try:
        h = h0.copy()
        run = oracle.run_dt if schedule == "double" else oracle.run
        lg = run(h, L, N, D, seed=seed, t0=0, n=n)
    finally:
        oracle.set_threads(0)
    return h, lg


def _same(g_log, r_log, g_h, r_h, what):
    for k, name in ((1, "s1"), (2, "s2"), (3, "accepted")):
        assert np.array_equal(g_log[name], r_log[:, k]), f"{what}: {name} differs"
    assert np.array_equal(g_h, r_h), f"{what}: heights differ"


# (L, N, D, seed, sweeps, start, packed, schedule)
KEYS = [
    (512, 2, 8, 3, 4, "rough", False, "checkerboard"),
    (2048, 1, 8, 5, 3, "flat", False, "checkerboard"),   # column-strip order offered
    (512, 4, 8, 7, 3, "cone", False, "checkerboard"),    # int8 blocks that need the wide path
    (1024, 1, 4, 9, 3, "rough", False, "checkerboard"),
    (1024, 3, 16, 11, 2, "rough", False, "checkerboard"),
    (512, 1, 2, 13, 3, "flat", False, "checkerboard"),
    (512, 2, 32, 15, 2, "rough", False, "checkerboard"),
    (1024, 2, 8, 17, 3, "rough", True, "checkerboard"),  # 16-bit storage
    (1024, 4, 8, 19, 3, "cone", True, "checkerboard"),   # 16-bit storage, wide path
    (1024, 1, 8, 21, 3, "rough", False, "double"),       # double tiling
]


def _start(L, N, seed, start):
    if start == "flat":
        return workloads.flat(L)
    if start == "cone":
        return workloads.cone(L, N, height=N * L // 4, seed=seed)
    return workloads.rough(L, min(N, 4), seed=seed)


@pytest.mark.parametrize("L,N,D,seed,sweeps,start,packed,schedule", KEYS)
def test_every_candidate_bit_exact(rsos, oracle, L, N, D, seed, sweeps, start, packed, schedule):
    from paper_1605_02620_amd import surface
    h0 = _start(L, N, seed, start)
    r_h, r_log = _oracle(oracle, h0, L, N, D, seed, sweeps, schedule)
    for batch in (False, True):
        cands = surface.tune_candidates(L, N, D, batch=batch, packed=packed, schedule=schedule)
        assert cands, "no candidate"
        for c in cands:
            c = dict(c, graph_sweeps=2)
            _say(f"L={L} N={N} D={D} packed={packed} {schedule} batch={batch} "
                 f"{c['TX']}x{c['TY']}x{c['NT']} elem={c['elem']} xmode={c['xmode']}")
            surface.tune_set(L, N, D, c, batch=batch, packed=packed, schedule=schedule)
            if not batch:
                s = rsos.Surface(L, N=N, seed=seed, D=D, h0=None if start == "flat" else h0, packed=packed,
                                 schedule=schedule, tune=True)
                s.sweep(sweeps)
                _same(s.log(1, sweeps), r_log, s.heights(), r_h, str(c))
                s.close()
            elif start == "flat":
                b = rsos.Batch([(L, N, seed)], D=D, packed=packed, schedule=schedule, tune=True)
                b.sweep(sweeps)
                _same(b.log(0, 1, sweeps), r_log, b.heights(0), r_h, str(c))
                b.close()
    surface.tune_clear()


def test_tuned_single_surface(rsos, oracle):
    """The configuration the tuner chooses for a 4096^2 surface (timed on
    this device) gives the oracle's bits."""
    from paper_1605_02620_amd import surface
    L, N, D, seed, n = 4096, 1, 8, 23, 3
    t = surface.tune(L, N, D)
    _say(f"tuned L={L}: {t}")
    assert t["measured"] == 1 and t["candidates"] >= 2 and t["ms_per_sweep"] > 0
    # the fastest candidate is never slower than the first fit; on a tie
    # within 1% the tuner takes the column-strip XCD order of the fastest
    # shape, which may then be up to 1% slower than the first fit
    slack = 1.01 if t["xmode"] == 2 else 1.0
    assert t["ms_per_sweep"] <= t["ms_first_fit"] * slack * 1.0001
    s = rsos.Surface(L, N=N, seed=seed, D=D, tune=True)
    s.sweep(n)
    r_h, r_log = _oracle(oracle, workloads.flat(L), L, N, D, seed, n)
    _same(s.log(1, n), r_log, s.heights(), r_h, f"tuned {t}")
    s.close()


def test_batch_with_several_kernel_instances(rsos, oracle):
    """A tuned batch whose (L, N) classes take different configurations runs
    one kernel instance per configuration in every sweep; every surface
    still gives the oracle's bits.  The configurations are forced so that
    they differ; a tuned mixed ensemble follows."""
    from paper_1605_02620_amd import surface
    specs = [(256, 1, 31), (512, 2, 32), (1024, 1, 33), (256, 1, 34), (512, 2, 35), (96, 1, 36)]
    forced = {(256, 1): dict(TX=16, TY=16, NT=256, elem=1, xmode=0, graph_sweeps=4),
              (512, 2): dict(TX=32, TY=8, NT=256, elem=1, xmode=1, graph_sweeps=4),
              (1024, 1): dict(TX=16, TY=8, NT=128, elem=4, xmode=1, graph_sweeps=4)}
    for (L, N), c in forced.items():
        surface.tune_set(L, N, 8, c, batch=True)
    n = 10
    os.environ["RSOS_BATCH_PLAN"] = "grouped"  # keep the three instances (no plan timing)
    try:
        b = rsos.Batch(specs, D=8, tune=True, stream=None)
    finally:
        del os.environ["RSOS_BATCH_PLAN"]
    b.sweep(n)
    for i, (L, N, seed) in enumerate(specs):
        r_h, r_log = _oracle(oracle, workloads.flat(L), L, N, 8, seed, n)
        _same(b.log(i, 1, n), r_log, b.heights(i), r_h, f"surface {i} L={L}")
    b.close()
    surface.tune_clear()
    # tuned (timed) choices for a mixed ensemble, uneven sweep counts; the
    # plan (grouped or one variant for all) is timed on the mix
    specs = [(256, 1, 40), (512, 1, 41), (1024, 2, 42), (2048, 1, 43)]
    counts = [7, 5, 6, 4]
    b = rsos.Batch(specs, D=8, tune=True)
    b.sweep(counts)
    for i, (L, N, seed) in enumerate(specs):
        r_h, r_log = _oracle(oracle, workloads.flat(L), L, N, 8, seed, counts[i])
        _same(b.log(i, 1, counts[i]), r_log, b.heights(i), r_h, f"tuned surface {i} L={L}")
    b.close()


def test_cache_round_trip(rsos, tmp_path):
    """The cache written to a file and read back gives the same choices
    without timing again."""
    from paper_1605_02620_amd import surface
    a = surface.tune(1024, 1, 8, batch=True)
    b = surface.tune(2048, 2, 8)
    path = tmp_path / "tune.txt"
    surface.tune_save(path)
    surface.tune_clear()
    surface.tune_load(path)
    a2 = surface.tune(1024, 1, 8, batch=True)
    b2 = surface.tune(2048, 2, 8)
    assert a2 == a and b2 == b
    surface.tune_clear()


def test_engine_with_tuned_choices(rsos, oracle):
    """Jobs served with per-class tuned configurations equal their oracle
    runs."""
    from paper_1605_02620_amd import serve
    eng = serve.Engine(pool_bytes=64 << 20, max_running=8, D=8, tune=True)
    jobs = [(256, 1, 51, 9), (512, 2, 52, 7), (1024, 1, 53, 5), (128, 1, 54, 6), (256, 4, 55, 8)]
    ids = [eng.submit(L, N, seed, t_max, sample_t=range(1, t_max + 1), keep_heights=True)
           for (L, N, seed, t_max) in jobs]
    while eng.stats()["running"] or eng.stats()["queued"]:
        eng.step(16)
    for jid, (L, N, seed, t_max) in zip(ids, jobs):
        samples, heights, _ = eng.result(jid, heights=True)
        r_h, r_log = _oracle(oracle, workloads.flat(L), L, N, 8, seed, t_max)
        _same(samples, r_log, heights, r_h, f"job L={L} N={N}")
    eng.close()
