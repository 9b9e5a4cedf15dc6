"""Steady-state finite-size-scaling workload (Sec. III.B and III.C).

Ensembles of surfaces of sizes L = 32..512 run in one batch to the steady
state; W is averaged over t >= t_start and over realizations; the direct fit
W_sat ~ L^alpha (Eq. (12)) and the effective exponents of Eq. (8) follow, and
the shape of the width and height distributions (Eqs. (13)-(15)) is measured
in the same window.

The onset of the steady state is estimated as in Eq. (7): a_N L^alpha =
b_N t^beta, with a_N and b_N deduced from small systems.  calibrate() fits
them on a pilot batch: b_N and beta from the early growth of W at the larger
pilot size, a_N and alpha from the plateaus of the pilot sizes.

Everything on the device is the library's batched path (rsos_batch_*): one
launch per sweep for the block-path sizes, one launch for all sweeps of the
LDS-resident sizes.  This module only schedules calls and reduces results.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import analysis
from .surface import Batch


def t_steady(L, a, b, alpha, beta):
    """Eq. (7): the time at which b t^beta reaches a L^alpha."""
    return (a * float(L) ** alpha / b) ** (1.0 / beta)


def _window_w(lg, t_from):
    """Time mean of W = sqrt(W^2) over the records with t >= t_from."""
    sel = lg["t"] >= t_from
    return float(np.sqrt(lg["w2"][sel]).mean())


def calibrate(N, D=8, sizes=(32, 64), realizations=16, growth=(8, 64), seed0=10_000,
              schedule="checkerboard"):
    """a_N, b_N, alpha and beta of Eq. (7) from a pilot batch of small
    systems run far into saturation (t = 40 L_max^1.62)."""
    t_run = int(40 * max(sizes) ** 1.62)
    specs = [(L, N, seed0 + k) for L in sizes for k in range(realizations)]
    b = Batch(specs, D=D, log_cap=t_run + 1, schedule=schedule)
    b.sweep(t_run)
    logs = [b.log(i, 1, t_run) for i in range(len(specs))]
    b.close()
    # growth: ensemble mean of W^2 at the larger pilot size, early times
    big = [lg for (L, _, _), lg in zip(specs, logs) if L == max(sizes)]
    t = big[0]["t"]
    w2 = np.mean([lg["w2"] for lg in big], axis=0)
    m = (t >= growth[0]) & (t <= growth[1])
    beta2, lnb2 = np.polyfit(np.log(t[m]), np.log(w2[m]), 1)
    beta, b_n = beta2 / 2.0, math.exp(lnb2 / 2.0)
    # plateaus: W averaged over the last half of the run
    wsat = [np.mean([_window_w(lg, t_run // 2) for (Ls, _, _), lg in zip(specs, logs) if Ls == L])
            for L in sizes]
    alpha, lna = analysis.power_fit(sizes, wsat)
    return {"a": math.exp(lna), "b": b_n, "alpha": alpha, "beta": beta}


def run(sizes=(32, 64, 128, 256, 512), N=1, realizations=32, D=8, start=2.0, window=2.0,
        moment_samples=32, calib=None, seed0=0, min_window=256, schedule="checkerboard"):
    """The steady-state workload.  Every size gets `realizations` surfaces
    (seeds seed0, seed0+1, ...); surface of size L runs to
    t_end = t_start + max(window t*, min_window) with t_start = start t*(L).
    Returns per-size W_sat (time and ensemble mean of W over t >= t_start,
    with its standard error over realizations), the W^2 and height shape
    statistics in the window, alpha_fit, and alpha_eff at the midpoints."""
    calib = calib or calibrate(N, D, schedule=schedule)
    sizes = sorted(int(L) for L in sizes)
    ts = {L: t_steady(L, **calib) for L in sizes}
    t_start = {L: int(math.ceil(start * ts[L])) for L in sizes}
    t_end = {L: t_start[L] + max(int(math.ceil(window * ts[L])), min_window) for L in sizes}
    specs = [(L, N, seed0 + k) for L in sizes for k in range(realizations)]
    ends = np.array([t_end[L] for (L, _, _) in specs], dtype=np.int64)
    log_cap = int(max(t_end[L] - t_start[L] for L in sizes)) + 2
    b = Batch(specs, D=D, log_cap=log_cap, schedule=schedule)
    # moment samples: evenly spaced in each size's window
    sample_t = {L: np.unique(np.linspace(t_start[L], t_end[L], moment_samples).astype(np.int64))
                for L in sizes}
    events = np.unique(np.concatenate([sample_t[L] for L in sizes] + [np.array([t_start[L] for L in sizes])]))
    moments = {L: [] for L in sizes}
    t = 0
    attempts = 0
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    for ev in events:
        steps = np.clip(np.minimum(ends, ev) - t, 0, None)
        if steps.max() > 0:
            b.sweep(steps)
            attempts += int(sum(int(st) * L * L for st, (L, _, _) in zip(steps, specs)))
        t = int(ev)
        for i, (L, _, _) in enumerate(specs):
            if t in sample_t[L]:
                moments[L].append(b.moments(i))
    rest = np.clip(ends - t, 0, None)
    if rest.max() > 0:
        b.sweep(rest)
        attempts += int(sum(int(st) * L * L for st, (L, _, _) in zip(rest, specs)))
    final = b.width()
    wall = time.perf_counter() - wall0
    per_size = {}
    for L in sizes:
        wmeans, w2s = [], []
        for i, (Ls, _, _) in enumerate(specs):
            if Ls != L:
                continue
            lg = b.log(i, t_start[L], t_end[L] - t_start[L] + 1)
            wmeans.append(_window_w(lg, t_start[L]))
            # W^2 samples for its distribution, thinned to one per t*/4
            stride = max(1, int(ts[L] / 4))
            w2s.extend(lg["w2"][::stride].tolist())
        s_w, q_w = analysis.shape(w2s)
        s_h, q_h = analysis.height_shape(moments[L])
        per_size[L] = {"t_steady": ts[L], "t_start": t_start[L], "t_end": t_end[L],
                       "W_sat": float(np.mean(wmeans)), "W_sat_err": analysis.stderr(wmeans),
                       "S_w2": s_w, "Q_w2": q_w, "S_h": s_h, "Q_h": q_h,
                       "w2_samples": len(w2s), "moment_samples": len(moments[L])}
    b.close()
    wsat = [per_size[L]["W_sat"] for L in sizes]
    alpha_fit, _ = analysis.power_fit(sizes, wsat)
    mid, a_eff = analysis.effective_exponent(sizes, wsat)
    return {"N": N, "D": D, "schedule": schedule, "realizations": realizations, "calibration": calib,
            "sizes": per_size, "alpha_fit": alpha_fit,
            "alpha_eff": [(float(x), float(y)) for x, y in zip(mid, a_eff)],
            "attempts": attempts, "wall_s": wall, "attempts_per_ns": attempts / (wall * 1e9),
            "final": [{"L": L, "seed": sd, "t": int(w["t"]), "s1": int(w["s1"]), "s2": int(w["s2"])}
                      for (L, _, sd), w in zip(specs, final)]}
