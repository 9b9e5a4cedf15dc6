"""Whole-run GPU parity against expected values that the CPU oracle wrote
(tests/golden/make_whole_runs.py, which calls only oracle/): every sweep's
(S1, S2, A) of Eq. (2) and the SHA-256 of the final heights, for the
growth runs of Sec. II / III.A at the workloads' full lengths, run the way
the benchmark runs them (non-default stream, hipGraph replays).

  single_L16384      L = 16384, N = 1, 2000 sweeps
  step_L8192_N*      L = 8192, N = 1, 2, 4, 5000 sweeps each
  ensemble_L*        the first surface of each size of the 256-surface
                     ensemble, 10^4 sweeps, run inside the whole ensemble
  served_subset      the served stream's jobs with L^2 t_max <= 2^29 plus a
                     seeded sample of larger ones, served together
  dt_L*_D*           the double-tiling schedule (Sec. II), 1000 sweeps,
                     L = 2048 with D = 8 and L = 1024 with D = 16
  ms_L*_N*           the multisurface lock-step mode, one group of 128
                     realizations: L = 256, N = 1 for 1000 sweeps and
                     L = 64, N = 8 for 2000 sweeps (the byte-staged kernel),
                     L = 64, N = 10 for 2000 sweeps (the 16-bit-staged one)

A run whose expected values have not been generated yet is skipped with
that reason.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "whole_runs")


def _say(msg):
    print(f"[whole-run] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rsos():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import paper_1605_02620_amd as pkg
    return pkg


def _gold(name):
    meta = os.path.join(GOLD, name + ".json")
    if not os.path.exists(meta):
        pytest.skip(f"{name}: expected values not generated (tests/golden/make_whole_runs.py {name})")
    return json.load(open(meta)), np.load(os.path.join(GOLD, name + ".npz"))


def _sha(h):
    return hashlib.sha256(np.ascontiguousarray(h, dtype="<i4").tobytes()).hexdigest()


def _check_log(lg, z, what):
    for name, key in (("s1", "s1"), ("s2", "s2"), ("accepted", "a")):
        bad = np.nonzero(lg[name] != z[key])[0]
        assert bad.size == 0, f"{what}: {name} differs first at t={int(bad[0]) + 1}"


def _single(rsos, name, packed=False):
    """One surface run whole in the benchmark's launch configuration (the
    autotuner's choice for its key)."""
    import torch
    meta, z = _gold(name)
    L, N, D, seed, n = meta["L"], meta["N"], meta["D"], meta["seed"], meta["sweeps"]
    sched = meta.get("schedule", "checkerboard")
    _say(f"{name}: L={L} N={N} D={D} seed={seed} sweeps={n} packed={packed} schedule={sched}")
    s = rsos.Surface(L, N=N, seed=seed, D=D, log_cap=n + 1, stream=torch.cuda.Stream(), packed=packed,
                     schedule=sched, tune=True)
    from paper_1605_02620_amd import surface
    c = surface.tune(L, N, D, packed=packed, schedule=sched)
    _say(f"{name}: {c['TX']}x{c['TY']} tiles, {c['NT']} threads, xmode {c['xmode']}, graphs of {c['graph_sweeps']}")
    s.sweep(n)
    lg = s.log(1, n)
    _check_log(lg, z, name)
    assert _sha(s.heights()) == meta["final_heights_sha256"], f"{name}: final heights differ"
    s.close()


def test_single_surface_whole_run(rsos):
    _single(rsos, "single_L16384")


def test_single_surface_whole_run_16bit_storage(rsos):
    _single(rsos, "single_L16384", packed=True)


@pytest.mark.parametrize("N", [1, 2, 4])
def test_step_heights_whole_run(rsos, N):
    _single(rsos, f"step_L8192_N{N}")


@pytest.mark.parametrize("N", [1, 2])
def test_step_heights_whole_run_16bit_storage(rsos, N):
    """The same runs with 16-bit residue storage (exact while N L <= 32766,
    so N = 4 at L = 8192 is outside it): the same expected values."""
    _single(rsos, f"step_L8192_N{N}", packed=True)


@pytest.mark.parametrize("packed,tune", [(False, False), (True, True)], ids=["int32", "16bit_tuned"])
def test_ensemble_whole_run(rsos, packed, tune):
    """The whole 256-surface ensemble in one batch for 10^4 sweeps (int32
    storage with the first-fit launch choice; 16-bit storage with the
    autotuner's per-class choices); the first surface of each size is
    compared sweep by sweep."""
    import torch
    ens = workloads.cfg_ensemble()
    names = {}
    for i, s in enumerate(ens):
        if s.L not in names:
            names[s.L] = i
    golds = {L: _gold(f"ensemble_L{L}") for L in names}
    n = ens[0].sweeps
    _say(f"ensemble: {len(ens)} surfaces, {n} sweeps, packed={packed}, tune={tune}")
    b = rsos.Batch([(s.L, s.N, s.seed) for s in ens], D=8, log_cap=n + 1, stream=torch.cuda.Stream(),
                   packed=packed, tune=tune)
    b.sweep(n)
    for L, i in names.items():
        meta, z = golds[L]
        assert (ens[i].seed, ens[i].N, n) == (meta["seed"], meta["N"], meta["sweeps"])
        _check_log(b.log(i, 1, n), z, f"ensemble surface {i} (L={L})")
        assert _sha(b.heights(i)) == meta["final_heights_sha256"], f"ensemble surface {i}: heights differ"
    b.close()


def test_served_subset_whole_runs(rsos):
    """The subset's jobs served together through the continuous-batching
    engine (all submitted at once; admission by footprint), each compared
    at its sample times and on its final heights."""
    from paper_1605_02620_amd import serve
    meta, z = _gold("served_subset")
    jobs = {j.job_id: j for j in workloads.job_stream(n_jobs=meta["stream"]["n_jobs"], rate_per_s=1.0,
                                                      seed=meta["stream"]["seed"])}
    ids = [int(i) for i in z["job_id"]]
    off = z["offsets"]
    _say(f"served subset: {len(ids)} jobs")
    eng = serve.Engine(pool_bytes=8 << 30, max_running=256, D=8)
    handle = {}
    for k, jid in enumerate(ids):
        j = jobs[jid]
        t = z["t"][off[k]:off[k + 1]]
        assert list(t) == workloads.pow2_grid(j.t_max)
        handle[jid] = eng.submit(j.L, j.N, j.seed, j.t_max, sample_t=t, keep_heights=True)
    while eng.stats()["running"] or eng.stats()["queued"]:
        eng.step(1 << 20)
    for k, jid in enumerate(ids):
        j = jobs[jid]
        samples, h, _ = eng.result(handle[jid], heights=True)
        sl = slice(off[k], off[k + 1])
        for name, key in (("s1", "s1"), ("s2", "s2"), ("accepted", "a")):
            assert np.array_equal(samples[name], z[key][sl]), f"job {jid} (L={j.L}, N={j.N}): {name} differs"
        assert _sha(h) == meta["final_heights_sha256"][str(jid)], f"job {jid}: final heights differ"
        eng.release(handle[jid])
    eng.close()


@pytest.mark.parametrize("name", ["dt_L2048_D8", "dt_L1024_D16"])
def test_double_tiling_whole_run(rsos, name):
    """The double-tiling schedule run whole (the autotuner's choice; this
    schedule runs with int32 storage only)."""
    _single(rsos, name)


@pytest.mark.parametrize("name", ["ms_L256_N1", "ms_L64_N8", "ms_L64_N10"])
def test_multisurface_whole_run(rsos, name):
    """One group of 128 lock-step realizations run whole: the SHA-256 of
    every realization's whole (S1, S2, A) log and of all final heights; the
    stored samples (every realization at every 100th sweep, the whole log
    of realizations 0-3) say where a difference starts."""
    import torch
    meta, z = _gold(name)
    L, N, seed, n = meta["L"], meta["N"], meta["seed"], meta["sweeps"]
    assert meta["D"] == 8 and meta["realizations"] == 128
    _say(f"{name}: L={L} N={N} seed={seed} sweeps={n}, 128 realizations")
    m = rsos.MultiSurface(L, N=N, seed=seed, groups=1, log_cap=n + 1, stream=torch.cuda.Stream())
    m.sweep(n)
    logs = [m.log(r, 1, n) for r in range(128)]
    for r in range(4):
        _check_log(logs[r], {k: z[k][r] for k in ("s1", "s2", "a")}, f"{name} realization {r}")
    ev = z["every"]
    for name_, key in (("s1", "s1_every"), ("s2", "s2_every"), ("accepted", "a_every")):
        got = np.stack([lg[name_][ev] for lg in logs])
        bad = np.argwhere(got != z[key])
        assert bad.size == 0, f"{name}: {name_} differs at realization {bad[0][0]}, t={int(ev[bad[0][1]]) + 1}"
    m_ = hashlib.sha256()
    for name_ in ("s1", "s2", "accepted"):
        m_.update(np.ascontiguousarray(np.stack([lg[name_] for lg in logs]), dtype="<i8").tobytes())
    assert m_.hexdigest() == meta["log_sha256"], f"{name}: whole logs differ"
    hs = np.stack([m.heights(r) for r in range(128)])
    assert _sha(hs) == meta["final_heights_sha256"], f"{name}: final heights differ"
    m.close()
