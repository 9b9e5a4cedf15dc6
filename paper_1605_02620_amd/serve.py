"""Continuous-batching job server over librsos.so's engine.

Argument marshalling plus the arrival loop: jobs are submitted when their
(wall-clock) arrival time comes, the engine admits them by device-memory
footprint as running jobs finish, and every running job advances one sweep
per tick.  Latency is measured from a job's arrival to the end of the chunk
in which it finished.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from ._lib import (JOB_CANCELLED, JOB_DONE, JOB_QUEUED, JOB_RUNNING, Params, Width, check, lib)
from .surface import LOG_DTYPE, _params, _require_gpu, _stream_handle, _widths

KEEP_HEIGHTS = 1


class Engine:
    def __init__(self, pool_bytes: int, max_running: int = 256, D: int = 8, device="cuda",
                 stream=None, tune: bool = False):
        dev = _require_gpu(device)
        self.D = int(D)
        self.stream = stream if stream is not None else torch.cuda.Stream(dev)
        self.pool = torch.empty(max(int(pool_bytes) // 4, 64), dtype=torch.int32, device=dev)
        self._h = ctypes.c_void_p()
        check(lib().rsos_engine_create(ctypes.byref(self._h), ctypes.c_void_p(self.pool.data_ptr()),
                                       self.pool.numel() * 4, int(max_running), self.D,
                                       _stream_handle(self.stream)))
        if tune:
            # per-class autotuned launch configurations (results unchanged)
            check(lib().rsos_engine_tune(self._h, 1))
        self._nsamples = {}

    def submit(self, L, N, seed, t_max, sample_t=(), keep_heights=False) -> int:
        st = np.ascontiguousarray(sorted(set(int(t) for t in sample_t)), dtype=np.int64)
        p = _params(L, N, self.D, seed)
        jid = ctypes.c_int64()
        check(lib().rsos_engine_submit(self._h, ctypes.byref(p), int(t_max),
                                       st.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), st.size,
                                       KEEP_HEIGHTS if keep_heights else 0, ctypes.byref(jid)))
        self._nsamples[jid.value] = (st.size, int(L))
        return jid.value

    def step(self, max_ticks: int = 16) -> int:
        n = ctypes.c_int32()
        check(lib().rsos_engine_step(self._h, int(max_ticks), ctypes.byref(n)))
        return n.value

    def poll(self, jid: int):
        s, t = ctypes.c_int32(), ctypes.c_int64()
        check(lib().rsos_engine_poll(self._h, int(jid), ctypes.byref(s), ctypes.byref(t)))
        return s.value, t.value

    def result(self, jid: int, heights: bool = False):
        n, L = self._nsamples[jid]
        buf = (Width * max(n, 1))()
        h = np.empty(L * L, dtype=np.int32) if heights else None
        lat = ctypes.c_double()
        check(lib().rsos_engine_result(self._h, int(jid), buf,
                                       h.ctypes.data_as(ctypes.c_void_p) if heights else None,
                                       ctypes.byref(lat)))
        return _widths(buf, n), h, lat.value

    def cancel(self, jid: int):
        check(lib().rsos_engine_cancel(self._h, int(jid)))

    def release(self, jid: int):
        check(lib().rsos_engine_release(self._h, int(jid)))
        self._nsamples.pop(jid, None)

    def stats(self) -> dict:
        a = (ctypes.c_int64 * 6)()
        check(lib().rsos_engine_stats(self._h, a))
        return dict(zip(("queued", "running", "finished", "bytes_in_use", "ticks", "attempts"), list(a)))

    def close(self):
        if self._h:
            check(lib().rsos_engine_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def serve(engine: Engine, jobs, chunk_ticks: int = 16, grid=None, keep_heights=False,
          time_limit_s: float | None = None, progress=None, progress_every_s: float = 30.0):
    """Runs a stream of jobs (objects with job_id, arrival_s, L, N, t_max,
    seed) through the engine in real time.  grid(t_max) gives each job's
    sample times; progress(message), if given, is called about every
    progress_every_s seconds.  Returns (per-job results dict, summary
    dict)."""
    order = sorted(jobs, key=lambda j: j.arrival_s)
    k = 0
    ids = {}
    delay = {}
    t0 = time.perf_counter()
    a0 = engine.stats()["attempts"]
    t_report = t0
    while True:
        now = time.perf_counter() - t0
        if progress is not None and time.perf_counter() - t_report > progress_every_s:
            t_report = time.perf_counter()
            st = engine.stats()
            progress(f"{now:.0f} s: {k} of {len(order)} jobs submitted, {st['running']} running, "
                     f"{st['queued']} queued")
        while k < len(order) and order[k].arrival_s <= now:
            j = order[k]
            gt = grid(j.t_max) if grid else [j.t_max]
            ids[j.job_id] = engine.submit(j.L, j.N, j.seed, j.t_max, gt, keep_heights)
            delay[j.job_id] = (time.perf_counter() - t0) - j.arrival_s
            k += 1
        st = engine.stats()
        if st["running"] == 0 and st["queued"] == 0:
            if k >= len(order):
                break
            time.sleep(max(0.0, order[k].arrival_s - (time.perf_counter() - t0)))
            continue
        engine.step(chunk_ticks)
        if time_limit_s is not None and time.perf_counter() - t0 > time_limit_s:
            break
    wall = time.perf_counter() - t0
    out = {}
    lat = []
    for j in order[:k]:
        jid = ids[j.job_id]
        state, _ = engine.poll(jid)
        if state != JOB_DONE:
            continue
        samples, h, lat_sub = engine.result(jid, heights=keep_heights)
        # latency from arrival: the driver's submission delay plus the engine's
        lat_arr = lat_sub + delay[j.job_id]
        out[j.job_id] = {"samples": samples, "heights": h, "latency_s": lat_arr}
        lat.append(lat_arr)
        engine.release(jid)
    attempts = engine.stats()["attempts"] - a0
    lat = np.asarray(lat) if lat else np.zeros(1)
    summary = {"jobs_done": len(out), "jobs_submitted": k, "wall_s": wall,
               "attempts": int(attempts), "attempts_per_ns": attempts / (wall * 1e9),
               "latency_p50_s": float(np.percentile(lat, 50)),
               "latency_p99_s": float(np.percentile(lat, 99))}
    return out, summary


__all__ = ["Engine", "serve", "JOB_QUEUED", "JOB_RUNNING", "JOB_DONE", "JOB_CANCELLED", "LOG_DTYPE"]
