#!/usr/bin/env python3
"""Writes the whole-run expected values of the large workloads, from the CPU
oracle only (oracle/ and the seeded input generators in workloads.py).

Each run starts flat (Sec. II) and follows the tile-checkerboard schedule
for its full length.  Stored per run:
  <name>.npz   int64 arrays s1, s2, a: S1 = sum h, S2 = sum h^2 and the
               accepted count A after every sweep t = 1 .. n (Eq. (2) needs
               S1, S2); served jobs keep only the records at their sample
               times (powers of two up to t_max, and t_max);
  <name>.json  parameters, the SHA-256 of the final int32 heights
               (little-endian, row-major) and of the stored arrays, the
               oracle's wall time and thread count.

Runs (names say what they are):
  single_L16384      L = 16384, N = 1, D = 8, seed 1, 2000 sweeps
  step_L8192_N{1,2,4}  L = 8192, N = 1, 2, 4, seed 1, 5000 sweeps
  ensemble_L{256,512,1024,2048}  the first surface of each size in the
               256-surface ensemble (its seed is its index), 10^4 sweeps
  served_subset      the served stream's jobs (2000 jobs, seed 5) with
               L^2 t_max <= 2^29, plus a seeded sample of 8 of the jobs with
               2^29 < L^2 t_max <= 2^33; each job alone
  dt_L2048_D8, dt_L1024_D16  the double-tiling schedule (Sec. II's four
               sets of sub-tiles), N = 1, seed 7, 1000 sweeps
  ms_L256_N1, ms_L64_N8, ms_L64_N10  the multisurface lock-step schedule,
               one group of 128 realizations (key = seed), seed 3, 1000,
               2000 and 2000 sweeps;
               stored: the whole log of realizations 0-3, every realization
               at every 100th sweep, and SHA-256s of the whole [128, n] log
               and of all final heights

Usage: python tests/golden/make_whole_runs.py [names...] [--threads 7]
Long runs checkpoint their state every 100 sweeps under --ckpt (default
/tmp/rsos_whole_run_ckpt) and resume from it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import ref  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(HERE, "whole_runs")
SUBSET_CAP = 2 ** 29
SAMPLE_CAP = 2 ** 33
SAMPLE_N = 8
SAMPLE_SEED = 1605


def sha_heights(h: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(h, dtype="<i4").tobytes()).hexdigest()


def sha_arrays(*arrs) -> str:
    m = hashlib.sha256()
    for a in arrs:
        m.update(np.ascontiguousarray(a, dtype="<i8").tobytes())
    return m.hexdigest()


def surfaces():
    """name -> (L, N, D, seed, sweeps)"""
    runs = {}
    c = workloads.cfg_single()
    runs["single_L16384"] = (c.L, c.N, c.D, c.seed, c.sweeps)
    for s in workloads.cfg_step_heights():
        runs[f"step_L8192_N{s.N}"] = (s.L, s.N, s.D, s.seed, s.sweeps)
    seen = set()
    for s in workloads.cfg_ensemble():
        if s.L not in seen:
            seen.add(s.L)
            runs[f"ensemble_L{s.L}"] = (s.L, s.N, s.D, s.seed, s.sweeps)
    return runs


DT_RUNS = {"dt_L2048_D8": (2048, 1, 8, 7, 1000), "dt_L1024_D16": (1024, 1, 16, 7, 1000)}
MS_RUNS = {"ms_L256_N1": (256, 1, 8, 3, 1000), "ms_L64_N8": (64, 8, 8, 3, 2000),
           "ms_L64_N10": (64, 10, 8, 3, 2000)}


def served_subset():
    """The served stream's jobs that the oracle runs whole: every job with
    L^2 t_max <= 2^29 and a seeded sample of larger ones."""
    jobs = workloads.job_stream(n_jobs=2000, rate_per_s=1.0, seed=5)
    work = [j.L * j.L * j.t_max for j in jobs]
    small = [j for j, w in zip(jobs, work) if w <= SUBSET_CAP]
    mid = [j for j, w in zip(jobs, work) if SUBSET_CAP < w <= SAMPLE_CAP]
    rng = np.random.default_rng(SAMPLE_SEED)
    pick = sorted(int(i) for i in rng.choice(len(mid), size=min(SAMPLE_N, len(mid)), replace=False))
    return small + [mid[i] for i in pick]


def run_surface(name, L, N, D, seed, n, threads, ckpt, schedule="checkerboard"):
    os.makedirs(ckpt, exist_ok=True)
    ck = os.path.join(ckpt, name + ".npz")
    ref.set_threads(threads)
    h = workloads.flat(L)
    done = 0
    logs = []
    if os.path.exists(ck):
        z = np.load(ck)
        h = np.ascontiguousarray(z["h"])
        logs = [z["log"]]
        done = int(z["done"])
        print(f"[{name}] resuming at t={done}", flush=True)
    t0 = time.perf_counter()
    step = 100
    while done < n:
        k = min(step, n - done)
        sweep = ref.run_dt if schedule == "double" else ref.run
        logs.append(sweep(h, L, N, D, seed=seed, t0=done, n=k))
        done += k
        np.savez(ck + ".tmp.npz", h=h, log=np.concatenate(logs), done=done)
        os.replace(ck + ".tmp.npz", ck)
        el = time.perf_counter() - t0
        print(f"[{name}] t={done}/{n}  {el:.0f} s", flush=True)
    lg = np.concatenate(logs)
    assert np.array_equal(lg[:, 0], np.arange(1, n + 1))
    s1, s2, a = (np.ascontiguousarray(lg[:, k]) for k in (1, 2, 3))
    np.savez_compressed(os.path.join(OUT, name + ".npz"), s1=s1, s2=s2, a=a)
    meta = {"name": name, "L": L, "N": N, "D": D, "seed": seed, "sweeps": n, "schedule": schedule,
            "final_heights_sha256": sha_heights(h), "log_sha256": sha_arrays(s1, s2, a),
            "final": {"s1": int(s1[-1]), "s2": int(s2[-1]), "a": int(a[-1])},
            "oracle_threads": threads, "oracle_wall_s": round(time.perf_counter() - t0, 1)}
    with open(os.path.join(OUT, name + ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    os.remove(ck)
    print(f"[{name}] written", flush=True)


def run_ms(name, L, N, D, seed, n, threads):
    ref.set_threads(threads)
    h = np.zeros((128, L * L), dtype=np.int32)
    t0 = time.perf_counter()
    lg = ref.run_ms(h, L, N, D, seed=seed, t0=0, n=n)
    assert np.array_equal(lg[0, :, 0], np.arange(1, n + 1))
    s1, s2, a = (np.ascontiguousarray(lg[:, :, k]) for k in (1, 2, 3))
    every = np.arange(99, n, 100)
    np.savez_compressed(os.path.join(OUT, name + ".npz"),
                        s1=s1[:4], s2=s2[:4], a=a[:4], every=every,
                        s1_every=np.ascontiguousarray(s1[:, every]),
                        s2_every=np.ascontiguousarray(s2[:, every]),
                        a_every=np.ascontiguousarray(a[:, every]))
    meta = {"name": name, "L": L, "N": N, "D": D, "seed": seed, "sweeps": n, "realizations": 128,
            "final_heights_sha256": sha_heights(h), "log_sha256": sha_arrays(s1, s2, a),
            "oracle_threads": threads, "oracle_wall_s": round(time.perf_counter() - t0, 1)}
    with open(os.path.join(OUT, name + ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(f"[{name}] written ({meta['oracle_wall_s']} s)", flush=True)


def _one_job(j):
    ref.set_threads(1)
    h = workloads.flat(j.L)
    lg = ref.run(h, j.L, j.N, j.D, seed=j.seed, t0=0, n=j.t_max)
    g = np.asarray(workloads.pow2_grid(j.t_max), dtype=np.int64)
    rec = lg[g - 1]
    return j.job_id, g, rec[:, 1].copy(), rec[:, 2].copy(), rec[:, 3].copy(), sha_heights(h)


def run_served(procs):
    jobs = served_subset()
    jobs.sort(key=lambda j: -j.L * j.L * j.t_max)  # longest first
    t0 = time.perf_counter()
    out = {}
    with mp.get_context("fork").Pool(procs) as pool:
        for k, r in enumerate(pool.imap_unordered(_one_job, jobs)):
            out[r[0]] = r
            if k % 25 == 0 or k == len(jobs) - 1:
                print(f"[served_subset] {k + 1}/{len(jobs)} jobs  {time.perf_counter() - t0:.0f} s", flush=True)
    ids = sorted(out)
    off = np.cumsum([0] + [len(out[i][1]) for i in ids]).astype(np.int64)
    cat = lambda k: np.concatenate([out[i][k] for i in ids]).astype(np.int64)  # noqa: E731
    t, s1, s2, a = cat(1), cat(2), cat(3), cat(4)
    np.savez_compressed(os.path.join(OUT, "served_subset.npz"), job_id=np.asarray(ids, dtype=np.int64),
                        offsets=off, t=t, s1=s1, s2=s2, a=a)
    meta = {"name": "served_subset", "stream": {"n_jobs": 2000, "seed": 5},
            "rule": f"L^2 t_max <= 2^29, plus {SAMPLE_N} jobs drawn with default_rng({SAMPLE_SEED}) "
                    "from those with 2^29 < L^2 t_max <= 2^33",
            "jobs": len(ids), "attempts": int(sum(j.L * j.L * j.t_max for j in jobs)),
            "final_heights_sha256": {str(i): out[i][5] for i in ids},
            "log_sha256": sha_arrays(t, s1, s2, a),
            "oracle_processes": procs, "oracle_wall_s": round(time.perf_counter() - t0, 1)}
    with open(os.path.join(OUT, "served_subset.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print("[served_subset] written", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*")
    ap.add_argument("--threads", type=int, default=7)
    ap.add_argument("--ckpt", default="/tmp/rsos_whole_run_ckpt")
    args = ap.parse_args()
    ref.build()
    os.makedirs(OUT, exist_ok=True)
    runs = surfaces()
    names = args.names or (["served_subset"] + [k for k in runs if k.startswith("ensemble")] +
                           ["single_L16384"] + [k for k in runs if k.startswith("step")])
    for nm in names:
        if nm == "served_subset":
            run_served(args.threads)
        elif nm in DT_RUNS:
            L, N, D, seed, n = DT_RUNS[nm]
            run_surface(nm, L, N, D, seed, n, args.threads, args.ckpt, schedule="double")
        elif nm in MS_RUNS:
            L, N, D, seed, n = MS_RUNS[nm]
            run_ms(nm, L, N, D, seed, n, args.threads)
        else:
            L, N, D, seed, n = runs[nm]
            run_surface(nm, L, N, D, seed, n, args.threads, args.ckpt)


if __name__ == "__main__":
    main()
