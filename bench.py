#!/usr/bin/env python3
"""Benchmark of the RSOS deposition sweep on one MI355X.

A step is one sweep (L^2 attempted depositions, both checkerboard phases and
the fused exact sums) of the single 16384^2 surface, N = 1, D = 8, flat
start, seed 1.  The timed region is K consecutive sweeps issued as one
rsos_sweep call, bracketed by device synchronisation; the lattice is already
resident in HBM when it starts.

Printed JSON line (one): attempts per ns over the timed region, plus
  roofline      the tile-block kernel's algorithmic HBM bytes (one read and
                one write of each int32 site per sweep: 8 B per attempt)
                divided by its mean duration, measured with HIP events on the
                surface's stream over the timed region, against 8 TB/s;
  cpu_baseline  the CPU oracle on a bounded sample of the same workload
                (a few sweeps of the same surface), all host cores;
  batched       the ensemble of 256 surfaces (L in {256..2048}) in one launch
                per sweep versus the same surfaces one surface per launch;
  served        a Poisson stream of jobs through the continuous-batching
                engine: p50/p99 latency from arrival and aggregate rate;
  packed16      the same surface and sweeps with heights kept on the device
                as 16-bit residues (identical results, 4 B per attempt), with
                its own roofline;
  moments       time of one exact height-distribution moment call on the
                final state (one read of the lattice);
  double_tiling the same surface under the paper's double-tiling schedule;
  multisurface  the lock-step multisurface mode against the batched path on
                the same 1024 realizations of L = 256;
  steady_state  a reduced run of the steady-state finite-size-scaling
                workload (L = 32..256).
--storage packed16 makes the 16-bit surface the headline (for profiling it
alone).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_ATTEMPT = 8  # int32 read + write per site per sweep


def _progress(msg):
    """One line per finished leg on stderr (the JSON result line is stdout's
    only line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _cores():
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(L, N, D, seed, budget_s=12.0):
    """The oracle as it stands, timed on the host on a few sweeps of the
    same surface (bounded to ~budget_s of CPU work)."""
    import numpy as np
    from oracle import ref
    import workloads
    # the host's usable cores, at most 16 (the share of the host that one GPU
    # of the benchmark machine comes with); both numbers are reported
    threads = min(_cores(), 16)
    ref.build()
    ref.set_threads(threads)
    h = workloads.flat(L)
    sweeps = 0
    t0 = time.perf_counter()
    while True:
        ref.run(h, L, N, D, seed=seed, t0=sweeps, n=1, log=False)
        sweeps += 1
        if time.perf_counter() - t0 > budget_s or sweeps >= 64:
            break
    dt = time.perf_counter() - t0
    # one thread, on the first sweeps of a smaller lattice of the same kind
    # (the per-attempt cost does not depend on L once the lattice outgrows
    # the caches)
    L1 = 4096
    ref.set_threads(1)
    h1 = workloads.flat(L1)
    n1 = 0
    t1 = time.perf_counter()
    while True:
        ref.run(h1, L1, N, D, seed=seed, t0=n1, n=1, log=False)
        n1 += 1
        if time.perf_counter() - t1 > budget_s / 4 or n1 >= 16:
            break
    dt1 = time.perf_counter() - t1
    ref.set_threads(0)
    return {"value": round(sweeps * L * L / (dt * 1e9), 4), "unit": "attempted site updates/ns",
            "cores": threads, "host_cores": _cores(), "kind": "oracle",
            "sample": f"first {sweeps} sweeps of the L={L} N={N} D={D} surface from flat, "
                      f"{dt:.1f} s, OpenMP over the tiles of a phase",
            "single_thread": {"value": round(n1 * L1 * L1 / (dt1 * 1e9), 4), "cores": 1,
                              "sample": f"first {n1} sweeps of an L={L1} N={N} D={D} surface "
                                        f"from flat, {dt1:.1f} s"}}


def kernel_instance(rocprof_name: str) -> str:
    from paper_1605_02620_amd import profiling
    return profiling.kernel_instance(rocprof_name)


def _traffic(kname, packed, schedule="checkerboard"):
    """Measured HBM bytes per launch from the committed counter summary, only
    while it describes this kernel source and instance."""
    from paper_1605_02620_amd import profiling
    if schedule == "double":
        name = "block_sweep_dt_traffic.json"
    else:
        name = "block_sweep16_traffic.json" if packed else "block_sweep_traffic.json"
    tr = profiling.current_traffic(os.path.join(ROOT, "profiles", name))
    if tr is not None and kernel_instance(tr.get("kernel", "")) == kname:
        return tr["traffic_bytes_per_launch"]
    return None


def bench_single(L, N, D, seed, steps, warmup, packed=False, schedule="checkerboard", tune=True):
    """K sweeps of one surface in one rsos_sweep call (hipGraph replays of
    one kernel per sweep), then the same again with every tile-block kernel
    timed by HIP events on the surface's stream that the runtime records at
    the kernel's start and end (graph replay off) for the dominant kernel's
    mean duration.  tune: the launch configuration
    comes from the autotuner (tuned when the surface is created)."""
    import torch
    import paper_1605_02620_amd as rsos
    stream = torch.cuda.Stream()
    s = rsos.Surface(L, N=N, seed=seed, D=D, log_cap=max(4096, steps + warmup + 1), stream=stream,
                     packed=packed, schedule=schedule, tune=tune)
    s.sweep(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.sweep(steps)
    s.width()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = L * L * steps / (dt * 1e9)
    s.timing(True)
    torch.cuda.synchronize()
    s.sweep(min(steps, 400))
    launches, mean_ms, _ = s.timing_read()
    s.timing(False)
    w = s.width()
    kname = s.kernel_name()
    # height-distribution moments of the final state (one read of the
    # lattice per call, synchronous)
    s.moments()
    t1 = time.perf_counter()
    for _ in range(10):
        mom = s.moments()
    mom_ms = (time.perf_counter() - t1) * 1e3 / 10
    s.close()
    bpa = BYTES_PER_ATTEMPT // 2 if packed else BYTES_PER_ATTEMPT
    achieved = L * L * bpa / (mean_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": _traffic(kname, packed, schedule), "traffic_unit": "bytes per launch",
                "kernel": kname, "launches_timed": launches, "kernel_mean_ms": round(mean_ms, 4),
                "algorithmic_bytes_per_launch": L * L * bpa}
    # the same bytes over the whole timed region (every launch and gap)
    roofline["frac_end_to_end"] = round(L * L * bpa * steps / dt / 1e9 / HBM_PEAK_GBS, 4)
    moments = {"ms_per_call": round(mom_ms, 4),
               "GBps_read": round(L * L * (bpa // 2) / (mom_ms * 1e-3) / 1e9, 1),
               "phi2": mom["phi2"], "phi3": mom["phi3"], "phi4": mom["phi4"]}
    out = {"value": value, "dt": dt, "w": w, "roofline": roofline, "moments": moments}
    if tune:
        from paper_1605_02620_amd import surface
        out["autotune"] = _tune_summary(surface.tune(L, N, D, packed=packed, schedule=schedule))
    return out


def _tune_summary(t):
    return {"shape": f"{t['TX']}x{t['TY']} tiles, {t['NT']} threads, {t['elem']}-byte staging",
            "xcd_order": {0: "in order", 1: "runs of 16 per XCD", 2: "column strips per XCD"}[t["xmode"]],
            "graph_sweeps": t["graph_sweeps"], "candidates": t["candidates"],
            "ms_per_sweep_tuned": round(t["ms_per_sweep"], 4),
            "ms_per_sweep_first_fit": round(t["ms_first_fit"], 4)}


def _run_batch(specs, sweeps, tune, warm=64):
    import torch
    import paper_1605_02620_amd as rsos
    b = rsos.Batch(specs, D=8, log_cap=sweeps + warm + 1, stream=torch.cuda.Stream(), tune=tune)
    b.sweep(warm)  # also builds the graphs the timed sweeps replay
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.sweep(sweeps)
    w = b.width()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.close()
    return dt, w


def bench_batched(sweeps=10000, plain_sweeps=1000):
    """The 256-surface ensemble (L from {256, 512, 1024, 2048}, N = 1):
    all surfaces swept together for its full 10^4 sweeps, with the
    autotuner's per-class configurations and with the untuned first-fit
    one; the plain one-surface-per-launch loop over the same surfaces for
    plain_sweeps sweeps each (its rate does not depend on the run length
    once the graphs are built)."""
    import torch
    import paper_1605_02620_amd as rsos
    import workloads
    ens = workloads.cfg_ensemble()
    specs = [(s.L, s.N, s.seed) for s in ens]
    total_sites = sum(L * L for (L, _, _) in specs)
    t_tuned, w_tuned = _run_batch(specs, sweeps, True)
    t_first, w_first = _run_batch(specs, sweeps, False)
    assert all(int(a) == int(b) for a, b in zip(w_tuned["s2"], w_first["s2"])), "tuned and first-fit runs differ"
    # plain: every surface its own handle, sweeps issued surface by surface
    warm = 64
    st = torch.cuda.Stream()
    surfs = [rsos.Surface(L, N=N, seed=sd, D=8, log_cap=plain_sweeps + warm + 1, stream=st, tune=True)
             for (L, N, sd) in specs]
    for s in surfs:
        s.sweep(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in surfs:
        s.sweep(plain_sweeps)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    for s in surfs:
        s.close()
    rate_b = total_sites * sweeps / (t_tuned * 1e9)
    rate_f = total_sites * sweeps / (t_first * 1e9)
    rate_p = total_sites * plain_sweeps / (tp * 1e9)
    return {"workload": "256 surfaces, L from {256,512,1024,2048} (default_rng(20160508)), "
                        f"N=1, D=8, seeds 0..255, {sweeps} sweeps each (batched); the plain loop "
                        f"times {plain_sweeps} sweeps per surface",
            "batched_attempts_per_ns": round(rate_b, 2),
            "batched_first_fit_attempts_per_ns": round(rate_f, 2),
            "tuned_over_first_fit": round(rate_b / rate_f, 3),
            "plain_attempts_per_ns": round(rate_p, 2), "batched_over_plain": round(rate_b / rate_p, 3),
            "batched_wall_s": round(t_tuned, 3)}


def bench_step_heights():
    """The step-height workload: three 8192^2 surfaces with N = 1, 2, 4,
    5000 sweeps each, one surface per launch (plain) and the three swept
    together (batched)."""
    import torch
    import paper_1605_02620_amd as rsos
    import workloads
    cfg = workloads.cfg_step_heights()
    n = cfg[0].sweeps
    sites = sum(c.L * c.L for c in cfg)
    st = torch.cuda.Stream()
    surfs = [rsos.Surface(c.L, N=c.N, seed=c.seed, D=c.D, log_cap=n + 65, stream=st, tune=True) for c in cfg]
    for s in surfs:
        s.sweep(64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in surfs:
        s.sweep(n)
    ws = [s.width() for s in surfs]
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    for s in surfs:
        s.close()
    tb, wb = _run_batch([(c.L, c.N, c.seed) for c in cfg], n, True)
    assert [int(w["s2"]) for w in ws] == [int(v) for v in wb["s2"]], "plain and batched runs differ"
    return {"workload": f"3 surfaces L=8192, N=1,2,4, D=8, seed 1, {n} sweeps each",
            "plain_attempts_per_ns": round(sites * n / (tp * 1e9), 2),
            "batched_attempts_per_ns": round(sites * n / (tb * 1e9), 2),
            "plain_wall_s": round(tp, 3),
            "W2_final": {int(c.N): round(float(w["w2"]), 4) for c, w in zip(cfg, ws)}}


def bench_multisurface(L=256, groups=8, sweeps=64):
    """Multisurface lock-step mode (groups of 128 realizations sharing a site
    sequence) against the batched path on the same realizations: aggregate
    attempted updates per ns (L^2 attempts per realization per sweep)."""
    import torch
    import paper_1605_02620_amd as rsos
    n_real = 128 * groups
    st = torch.cuda.Stream()
    # the warm-up also builds the graphs the timed sweeps replay
    warm = 64
    m = rsos.MultiSurface(L, N=1, seed=1, groups=groups, log_cap=sweeps + warm + 8, stream=st)
    m.sweep(warm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    m.sweep(sweeps)
    m.log(0, sweeps + warm, 1)
    torch.cuda.synchronize()
    t_ms = time.perf_counter() - t0
    m.close()
    t_b = {}
    for packed in (False, True):
        b = rsos.Batch([(L, 1, k) for k in range(n_real)], D=8, log_cap=sweeps + warm + 8, stream=st,
                       packed=packed)
        b.sweep(warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.sweep(sweeps)
        b.log(0, sweeps + warm, 1)
        torch.cuda.synchronize()
        t_b[packed] = time.perf_counter() - t0
        b.close()
    work = n_real * L * L * sweeps
    return {"workload": f"{n_real} realizations of L={L}, N=1, D=8, {sweeps} sweeps",
            "multisurface_attempts_per_ns": round(work / (t_ms * 1e9), 2),
            "batched_attempts_per_ns": round(work / (t_b[False] * 1e9), 2),
            "batched_packed16_attempts_per_ns": round(work / (t_b[True] * 1e9), 2)}


def bench_fss(sizes=(32, 64, 128, 256), realizations=256):
    """Reduced steady-state finite-size-scaling run (the paper's second
    workload at L = 32..256): aggregate rate and the fitted exponent."""
    from paper_1605_02620_amd import fss
    r = fss.run(sizes=sizes, N=1, realizations=realizations, start=2.0, window=4.0, moment_samples=16)
    return {"workload": f"L in {list(sizes)}, N=1, D=8, {realizations} realizations each, "
                        "t_start = 2 t*, window 4 t* (t* from Eq. (7) calibrated on L = 32, 64)",
            "attempts_per_ns": round(r["attempts_per_ns"], 2), "wall_s": round(r["wall_s"], 2),
            "alpha_fit": round(r["alpha_fit"], 4),
            "W_sat": {int(L): round(v["W_sat"], 4) for L, v in r["sizes"].items()},
            "S_w2": {int(L): round(v["S_w2"], 3) for L, v in r["sizes"].items()},
            "S_h": {int(L): round(v["S_h"], 3) for L, v in r["sizes"].items()},
            "Q_h": {int(L): round(v["Q_h"], 3) for L, v in r["sizes"].items()}}


def served_jobs(n_jobs):
    """The first n_jobs jobs of the served stream (2000 jobs, default_rng(5):
    L = 2^7..2^13, N in {1, 2, 4}, t_max log-uniform in [100, 20000])."""
    import workloads
    return workloads.job_stream(n_jobs=2000, rate_per_s=1.0, seed=5)[:n_jobs]


def bench_plain_jobs(jobs):
    """The plain one-surface-per-launch loop over a job set: each job alone,
    one after the other, on one stream; aggregate attempted updates/ns."""
    import torch
    import paper_1605_02620_amd as rsos
    import workloads
    st = torch.cuda.Stream()
    attempts = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_report = t0
    for i, j in enumerate(jobs):
        s = rsos.Surface(j.L, N=j.N, seed=j.seed, D=8, log_cap=j.t_max + 1, stream=st, tune=True)
        s.sweep(j.t_max)
        s.log(1, j.t_max)  # the job's records (synchronises)
        s.close()
        attempts += j.L * j.L * j.t_max
        if time.perf_counter() - t_report > 30.0:
            t_report = time.perf_counter()
            _progress(f"served: plain loop, {i + 1} of {len(jobs)} jobs")
    dt = time.perf_counter() - t0
    return attempts / (dt * 1e9), dt


def bench_served(jobs, rate_attempts_per_ns=None, load=0.9, pool_gib=8, tune=True):
    """The jobs through the continuous-batching engine: as a Poisson stream
    at `load` times the given rate (attempted updates per ns), or all
    arriving at once (rate None: the engine's capacity on this job set);
    p50/p99 latency from arrival and aggregate attempted updates/ns."""
    import numpy as np
    import torch
    from paper_1605_02620_amd import serve
    import workloads
    if rate_attempts_per_ns is None:
        arr = np.zeros(len(jobs))
        rate = None
    else:
        mean_attempts = float(np.mean([j.L * j.L * j.t_max for j in jobs]))
        rate = load * rate_attempts_per_ns * 1e9 / mean_attempts  # jobs per second
        rng = np.random.default_rng(55)
        gaps = rng.exponential(1.0 / rate, size=len(jobs))
        arr = np.cumsum(gaps) - gaps[0]
    timed = [workloads.Job(job_id=j.job_id, arrival_s=float(a), L=j.L, N=j.N, t_max=j.t_max, seed=j.seed)
             for j, a in zip(jobs, arr)]
    eng = serve.Engine(pool_bytes=pool_gib << 30, max_running=256, D=8, tune=tune)
    res, summ = serve.serve(eng, timed, grid=lambda tm: workloads.pow2_grid(tm),
                            progress=lambda m: _progress(f"served: {m}"))
    eng.close()
    torch.cuda.synchronize()
    out = {"jobs_done": summ["jobs_done"], "wall_s": round(summ["wall_s"], 3),
           "attempts_per_ns": round(summ["attempts_per_ns"], 2),
           "latency_p50_s": round(summ["latency_p50_s"], 4),
           "latency_p99_s": round(summ["latency_p99_s"], 4)}
    if rate is not None:
        out["arrival_rate_per_s"] = round(rate, 3)
    return out


SERVED_LOADS = ("0.9", "0.9ff", "0.5")


def bench_serving(n_jobs, loads=SERVED_LOADS):
    """Served against plain on the same jobs.  The autotuner's choices for
    every (L, N) class of the job set are made first (setup, outside every
    timed region).  capacity: all jobs arrive at once; then Poisson streams
    at 0.9 and 0.5 of that capacity (latency from arrival), and at 0.9 with
    the untuned first-fit launch choice ("0.9ff"), as many of them as
    `loads` names."""
    from paper_1605_02620_amd import surface
    jobs = served_jobs(n_jobs)
    for (L, N) in sorted({(j.L, j.N) for j in jobs}):
        if L * L * 4 > 64 * 1024:
            surface.tune(L, N, 8, batch=True)
            surface.tune(L, N, 8)
    plain_rate, plain_s = bench_plain_jobs(jobs)
    _progress(f"served: plain loop {plain_rate:.1f} attempts/ns")
    full = n_jobs >= 2000
    out = {"workload": (f"{'all' if full else 'the first'} {n_jobs} jobs of the served stream (2000 jobs, "
                        "default_rng(5): L = 2^7..2^13, N in {1,2,4}, t_max log-uniform in [100, 20000]), "
                        "8 GiB pool" + ("" if full else "; reduced from the full 2000-job stream to keep the "
                                                        "default run short")),
           "attempts": int(sum(j.L * j.L * j.t_max for j in jobs)),
           "plain_attempts_per_ns": round(plain_rate, 2), "plain_wall_s": round(plain_s, 3)}
    cap = bench_served(jobs)
    out["capacity"] = cap
    out["served_over_plain"] = round(cap["attempts_per_ns"] / plain_rate, 3)
    _progress(f"served: capacity {cap['attempts_per_ns']} attempts/ns")
    if "0.9" in loads:
        out["at_0.9_load"] = bench_served(jobs, cap["attempts_per_ns"], 0.9)
        _progress("served: 0.9 load done")
    if "0.9ff" in loads:
        out["at_0.9_load_first_fit"] = bench_served(jobs, cap["attempts_per_ns"], 0.9, tune=False)
        _progress("served: 0.9 load, first fit, done")
    if "0.5" in loads:
        out["at_0.5_load"] = bench_served(jobs, cap["attempts_per_ns"], 0.5)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=64)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-stream leg")
    ap.add_argument("--no-packed", action="store_true", help="skip the 16-bit storage leg")
    ap.add_argument("--no-ms", action="store_true", help="skip the multisurface leg")
    ap.add_argument("--no-dt", action="store_true", help="skip the double-tiling leg")
    ap.add_argument("--no-fss", action="store_true", help="skip the steady-state leg")
    ap.add_argument("--storage", choices=("int32", "packed16"), default="int32",
                    help="height storage of the headline surface")
    ap.add_argument("--schedule", choices=("checkerboard", "double"), default="checkerboard",
                    help="tile schedule of the headline surface (the double-tiling leg uses 'double')")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (calibrates HBM counters)")
    ap.add_argument("--no-step", action="store_true", help="skip the step-height leg")
    ap.add_argument("--served-jobs", type=int, default=200,
                    help="jobs of the 2000-job served stream to serve (2000: the whole stream)")
    ap.add_argument("--served-loads", default=",".join(SERVED_LOADS),
                    help="comma-separated Poisson loads served after the capacity run: "
                         "0.9, 0.9ff (0.9 with the untuned first-fit choice), 0.5")
    ap.add_argument("--no-tune", action="store_true", help="headline without the autotuner")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file: read before the run if it exists, written after the "
                         "headline (profiling runs reuse the choices without timing candidates)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(independent surfaces shard across GPUs without communication)", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads

    cfg = workloads.cfg_single()
    L, N, D, seed = cfg.L, cfg.N, cfg.D, cfg.seed
    if args.tune_cache and os.path.exists(args.tune_cache):
        from paper_1605_02620_amd import surface
        surface.tune_load(args.tune_cache)
    head = bench_single(L, N, D, seed, args.steps, args.warmup, packed=args.storage == "packed16",
                        schedule=args.schedule, tune=not args.no_tune)
    value, dt, w, roofline = head["value"], head["dt"], head["w"], head["roofline"]
    if args.tune_cache:
        from paper_1605_02620_amd import surface
        surface.tune_save(args.tune_cache)
    _progress(f"headline: {value:.1f} attempts/ns")
    out = {"metric": "attempted site updates/ns", "value": round(value, 3),
           "unit": "attempts/ns", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(dt * 1e3 / args.steps, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
           "config": {"workload": f"single RSOS surface L={L} periodic, N={N}, D={D}, flat int32 "
                                  f"start, seed {seed}, {args.steps} sweeps timed after "
                                  f"{args.warmup} warm-up sweeps",
                      "L": L, "N": N, "D": D, "seed": seed, "sweeps": args.steps,
                      "storage": args.storage, "schedule": args.schedule,
                      "final_t": int(w["t"]), "final_w2": float(w["w2"])},
           "roofline": roofline, "moments": head["moments"]}
    if "autotune" in head:
        out["autotune"] = head["autotune"]
    if args.storage == "int32" and args.schedule == "checkerboard" and not args.no_packed:
        # the same surface and sweeps with heights kept as 16-bit residues
        # (identical results; 4 B per attempt)
        pk = bench_single(L, N, D, seed, args.steps, args.warmup, packed=True)
        out["packed16"] = {"value": round(pk["value"], 3), "unit": "attempts/ns",
                           "ms_per_step": round(pk["dt"] * 1e3 / args.steps, 4),
                           "final_t": int(pk["w"]["t"]), "final_w2": float(pk["w"]["w2"]),
                           "same_result": bool(pk["w"]["s1"] == w["s1"] and pk["w"]["s2"] == w["s2"]),
                           "roofline": pk["roofline"], "moments": pk["moments"]}
    if args.copy_probe:
        src = torch.ones(L * L, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_probe"] = {"bytes_each": 2 * src.numel() * 4, "copies": 5,
                             "GBps": round(5 * 2 * src.numel() * 4 / (time.perf_counter() - t0) / 1e9, 1)}
        del src, dst
    if not args.no_batch:
        out["batched"] = bench_batched()
        _progress(f"batched: {out['batched']['batched_attempts_per_ns']} attempts/ns")
    if not args.no_step:
        out["step_heights"] = bench_step_heights()
        _progress("step heights done")
    if not args.no_dt:
        # the paper's double-tiling schedule on the same surface (a different
        # but equally valid dynamics; same 8 B per attempt)
        dt_steps = min(args.steps, 400)
        dtr = bench_single(L, N, D, seed, dt_steps, args.warmup, schedule="double")
        out["double_tiling"] = {"value": round(dtr["value"], 3), "unit": "attempts/ns",
                                "ms_per_step": round(dtr["dt"] * 1e3 / dt_steps, 4), "sweeps": dt_steps,
                                "roofline": dtr["roofline"]}
    if not args.no_ms:
        out["multisurface"] = bench_multisurface()
        _progress("multisurface done")
    if not args.no_fss:
        out["steady_state"] = bench_fss()
        _progress("steady state done")
    if not args.no_serve:
        out["served"] = bench_serving(args.served_jobs, tuple(x for x in args.served_loads.split(",") if x))
        _progress("served done")
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(L, N, D, seed)
        _progress("cpu baseline done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
