"""GPU checks at the full shapes of the step-height, ensemble and served
workloads, in the launch configurations that run them.

The oracle computes the first sweeps of every sampled surface bit for bit;
whole runs are checked through properties that hold at any size: the
restriction of Sec. I on every bond, S1 equal to the accepted-deposit
ledger, S2 equal to the sum of squared heights, and KPZ growth of W^2
(beta near 0.24, Sec. III.A).
"""
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[configs] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rsos():
    import torch
    assert torch.cuda.is_available()
    import paper_1605_02620_amd as p
    return p


def _properties(h, log, L, N):
    h = h.reshape(L, L).astype(np.int64)
    assert np.abs(h - np.roll(h, 1, axis=0)).max() <= N
    assert np.abs(h - np.roll(h, 1, axis=1)).max() <= N
    assert int(log["s1"][-1]) == int(log["accepted"].sum()) == int(h.sum())
    assert int(log["s2"][-1]) == int((h * h).sum())


def _oracle_first(oracle, L, N, D, seed, n):
    oracle.set_threads(16)
    try:
        h = workloads.flat(L)
        lg = oracle.run(h, L, N, D, seed=seed, t0=0, n=n)
    finally:
        oracle.set_threads(0)
    return h, lg


def test_step_heights_first_sweeps_and_full_run(rsos, oracle):
    """Three L = 8192 surfaces, N = 1, 2, 4, seed 1: batched together; the
    first 3 sweeps bit for bit against the oracle, then 5000 sweeps."""
    cfgs = workloads.cfg_step_heights()
    specs = [(c.L, c.N, c.seed) for c in cfgs]
    _say(f"step heights {specs}")
    b = rsos.Batch(specs, D=8)
    b.sweep(3)
    for i, c in enumerate(cfgs):
        r_h, r_log = _oracle_first(oracle, c.L, c.N, c.D, c.seed, 3)
        g_log = b.log(i, 1, 3)
        assert np.array_equal(b.heights(i), r_h)
        for k, name in ((1, "s1"), (2, "s2"), (3, "accepted")):
            assert np.array_equal(g_log[name], r_log[:, k])
    b.sweep(cfgs[0].sweeps - 3)
    for i, c in enumerate(cfgs):
        lg = b.log(i, 1, c.sweeps)
        _properties(b.heights(i), lg, c.L, c.N)
        ts = lg["t"].astype(float)
        m = (ts >= 100) & (ts <= 5000)
        beta = np.polyfit(np.log(ts[m]), np.log(lg["w2"][m]), 1)[0] / 2
        _say(f"N={c.N} beta(100..5000) = {beta:.4f}")
        assert 0.2 <= beta <= 0.27


def test_ensemble_full_shape(rsos, oracle):
    """256 surfaces, L from {256, 512, 1024, 2048}, seeds 0..255, one launch
    per sweep: a sample of surfaces bit for bit over their first sweeps
    (every L present), then 10000 sweeps with properties on all surfaces."""
    ens = workloads.cfg_ensemble()
    specs = [(s.L, s.N, s.seed) for s in ens]
    _say("ensemble 256 surfaces")
    b = rsos.Batch(specs, D=8, log_cap=16384)
    n0 = 8
    b.sweep(n0)
    picked = {}
    for i, s in enumerate(ens):
        picked.setdefault(s.L, i)
    for L, i in sorted(picked.items()):
        r_h, r_log = _oracle_first(oracle, L, 1, 8, ens[i].seed, n0)
        assert np.array_equal(b.heights(i), r_h), f"surface {i} (L={L})"
        assert np.array_equal(b.log(i, 1, n0)["s2"], r_log[:, 2])
    b.sweep(ens[0].sweeps - n0)
    w = b.width()
    assert all(int(x) == ens[0].sweeps for x in w["t"])
    for i, s in enumerate(ens):
        lg = b.log(i, 1, s.sweeps)
        _properties(b.heights(i), lg, s.L, s.N)
    # ensemble means of W^2 per L at the last sweep: finite, ordered by L
    # while the smaller systems saturate (t_x ~ L^1.6)
    means = {L: float(np.mean([w["w2"][i] for i, s in enumerate(ens) if s.L == L])) for L in picked}
    _say(f"<W^2>(t=10^4) by L: {means}")
    assert means[256] < means[2048]


def test_served_stream_matches_alone(rsos, oracle):
    """A served stream with the job mix of the serving workload (L a power
    of two in [128, 8192], N in {1, 2, 4}, log-uniform t_max) scaled to
    short runs: every job equals its solo run; the smallest few also equal
    the oracle."""
    from paper_1605_02620_amd import serve
    jobs = workloads.job_stream(n_jobs=24, rate_per_s=400.0, seed=5, t_range=(20, 200))
    eng = serve.Engine(pool_bytes=2 << 30, max_running=16, D=8)
    res, summ = serve.serve(eng, jobs, keep_heights=True,
                            grid=lambda tm: workloads.pow2_grid(tm))
    _say(f"served summary {summ}")
    assert summ["jobs_done"] == len(jobs)
    for j in sorted(jobs, key=lambda j: j.L * j.L * j.t_max):
        alone = rsos.Surface(j.L, N=j.N, seed=j.seed, D=8)
        alone.sweep(j.t_max)
        assert np.array_equal(res[j.job_id]["heights"], alone.heights()), f"job {j.job_id}"
        lg = alone.log(1, j.t_max)
        for rec in res[j.job_id]["samples"]:
            t = int(rec["t"])
            assert (rec["s1"], rec["s2"]) == (lg["s1"][t - 1], lg["s2"][t - 1])
        alone.close()
    for j in sorted(jobs, key=lambda j: j.L * j.L * j.t_max)[:4]:
        r_h, _ = _oracle_first(oracle, j.L, j.N, 8, j.seed, j.t_max)
        assert np.array_equal(res[j.job_id]["heights"], r_h)
    eng.close()
