"""Seeded synthetic inputs for the RSOS deposition sweep.

This module is the only code shared by the GPU path's tests/benchmarks and
the CPU oracle: it generates inputs (lattice sizes, restrictions, seeds,
initial surfaces, sample-time grids and job streams) and holds none of the
model's arithmetic.  The paper (Kelling, Odor & Gemming) simulates from flat
initial conditions with restriction N = 1, 3, 5, 7 on L = 4096 .. 9605
(Sec. II) and measures steady states for L = 32 .. 512 (Sec. III.B); the
configurations here are scaled versions of those workloads.  No dataset is
involved: everything is generated from the seeds below.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


# --------------------------------------------------------------------------
# initial surfaces
# --------------------------------------------------------------------------
def flat(L: int) -> np.ndarray:
    """Flat initial condition h = 0 (Sec. II)."""
    return np.zeros(L * L, dtype=np.int32)


def _closed_walk(rng, n: int, N: int) -> np.ndarray:
    """A periodic integer walk of n steps in [-N, N] that returns to its start."""
    steps = rng.integers(-N, N + 1, size=n)
    # repair the total to zero by moving single steps toward zero
    total = int(steps.sum())
    idx = rng.permutation(n)
    k = 0
    while total != 0:
        i = idx[k % n]
        if total > 0 and steps[i] > -N:
            steps[i] -= 1
            total -= 1
        elif total < 0 and steps[i] < N:
            steps[i] += 1
            total += 1
        k += 1
    walk = np.concatenate([[0], np.cumsum(steps)[:-1]])
    return walk.astype(np.int64)


def rough(L: int, N: int, seed: int, base: int = 0, amp: int | None = None) -> np.ndarray:
    """A seeded rough surface that satisfies |h_i - h_j| <= N on every bond.

    h(x, y) = base + f(x) + g(y) with f, g closed periodic walks whose steps
    lie in [-a, a], a = N unless `amp` is smaller, shifted so that min h =
    base.  A bond along x sees only a step of f, one along y only a step of g."""
    rng = np.random.default_rng(seed)
    a = N if amp is None else amp
    a = max(0, min(a, N))
    f = _closed_walk(rng, L, a) if a > 0 else np.zeros(L, dtype=np.int64)
    g = _closed_walk(rng, L, a) if a > 0 else np.zeros(L, dtype=np.int64)
    h = f[None, :] + g[:, None]
    h = h - h.min() + base
    return np.ascontiguousarray(h.reshape(-1).astype(np.int32))


def cone(L: int, N: int, height: int, seed: int = 0) -> np.ndarray:
    """A Manhattan cone h = max(0, height - N |x - cx| - N |y - cy|) around a
    seeded centre (periodic distance): every bond differs by at most N, steep
    near the apex and flat far from it."""
    rng = np.random.default_rng(seed)
    cx, cy = (int(v) for v in rng.integers(0, L, size=2))
    x = np.arange(L)
    dx = np.minimum((x - cx) % L, (cx - x) % L)
    dy = np.minimum((x - cy) % L, (cy - x) % L)
    h = np.maximum(0, height - N * (dx[None, :] + dy[:, None]))
    return np.ascontiguousarray(h.reshape(-1).astype(np.int32))


def violating(L: int, N: int, seed: int) -> np.ndarray:
    """A surface with exactly one bond whose height difference exceeds N."""
    rng = np.random.default_rng(seed)
    h = flat(L)
    x, y = (int(v) for v in rng.integers(0, L, size=2))
    h[y * L + x] = N + 1
    return h


# --------------------------------------------------------------------------
# sample-time grids
# --------------------------------------------------------------------------
def pow2_grid(t_max: int, include_end: bool = True) -> list[int]:
    g = [1 << k for k in range(0, 63) if (1 << k) <= t_max]
    if include_end and g[-1] != t_max:
        g.append(t_max)
    return g


def log_grid(t_max: int, n: int = 64) -> list[int]:
    """n log-spaced integer times t_k = max(t_{k-1} + 1, round(t_max^(k/(n-1))))."""
    out = []
    prev = 0
    for k in range(n):
        t = max(prev + 1, int(round(t_max ** (k / (n - 1)))))
        t = min(t, t_max)
        if out and t == out[-1]:
            continue
        out.append(t)
        prev = t
    if out[-1] != t_max:
        out.append(t_max)
    return out


def paper_grid(t_max: float, m: float = 0.01, t0: float = 0.0) -> list[int]:
    """Measurement times of Eq. (10), t_{i+1} = (t_i + 10) e^m from t_0, rounded
    to integers (the rounding is not stated in the paper) and de-duplicated."""
    out = []
    t = t0
    while True:
        t = (t + 10.0) * math.exp(m)
        if t > t_max:
            break
        ti = int(round(t))
        if not out or ti != out[-1]:
            out.append(ti)
    return out


# --------------------------------------------------------------------------
# benchmark / parity configurations
# --------------------------------------------------------------------------
@dataclass
class Surface:
    L: int
    N: int
    seed: int
    sweeps: int
    D: int = 8
    grid: list[int] = field(default_factory=list)


def cfg_small() -> Surface:
    """L = 64, N = 1, seed 1, flat; 1024 sweeps so that W^2 can be read at
    t = 2^0 .. 2^10 and at t = 1000."""
    return Surface(L=64, N=1, seed=1, sweeps=1024, grid=sorted(set(pow2_grid(1024) + [1000])))


def cfg_single() -> Surface:
    """The single large surface: L = 16384, N = 1, seed 1, flat, 2000 sweeps."""
    return Surface(L=16384, N=1, seed=1, sweeps=2000, grid=pow2_grid(2000))


def cfg_step_heights() -> list[Surface]:
    """Three L = 8192 surfaces with N = 1, 2, 4, seed 1 each, 5000 sweeps."""
    return [Surface(L=8192, N=n, seed=1, sweeps=5000, grid=log_grid(5000)) for n in (1, 2, 4)]


def cfg_ensemble(n: int = 256, sweeps: int = 10000) -> list[Surface]:
    """256 independent surfaces, L drawn from {256, 512, 1024, 2048} with
    numpy default_rng(20160508), N = 1, seeds 0..255, flat."""
    rng = np.random.default_rng(20160508)
    Ls = rng.choice([256, 512, 1024, 2048], size=n)
    return [Surface(L=int(L), N=1, seed=i, sweeps=sweeps, grid=log_grid(sweeps))
            for i, L in enumerate(Ls)]


@dataclass
class Job:
    job_id: int
    arrival_s: float
    L: int
    N: int
    t_max: int
    seed: int
    D: int = 8


def job_stream(n_jobs: int = 2000, rate_per_s: float = 10.0, seed: int = 5,
               L_pow=(7, 13), Ns=(1, 2, 4), t_range=(100, 20000)) -> list[Job]:
    """Poisson arrivals: exponential inter-arrival times at `rate_per_s`;
    L uniform over the powers of two 2^L_pow[0] .. 2^L_pow[1]; N uniform over
    Ns; t_max = round(exp(U[ln t_lo, ln t_hi])); 64-bit random seeds."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_jobs)
    arr = np.cumsum(gaps) - gaps[0]
    Ls = 2 ** rng.integers(L_pow[0], L_pow[1] + 1, size=n_jobs)
    Nv = rng.choice(np.asarray(Ns), size=n_jobs)
    tm = np.rint(np.exp(rng.uniform(math.log(t_range[0]), math.log(t_range[1]), size=n_jobs)))
    seeds = rng.integers(0, 2 ** 63, size=n_jobs, dtype=np.int64).astype(np.uint64)
    return [Job(job_id=i, arrival_s=float(arr[i]), L=int(Ls[i]), N=int(Nv[i]), t_max=int(tm[i]),
                seed=int(seeds[i])) for i in range(n_jobs)]
