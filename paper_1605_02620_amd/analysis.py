"""Host-side statistics over the library's exact per-sweep records.

These are the estimators the paper applies to its samples; they run on the
host over results the GPU path has produced (W^2 records, moment records).

  shape(values)          skewness and kurtosis of a sample (Eqs. (13)-(15)
                         applied to one observable, e.g. W^2)
  height_shape(records)  S_h and Q_h from per-state height moments: ratios
                         of sample averages of Phi_3, Phi_4 and Phi_2
  effective_exponent     local slopes of Eq. (8) between consecutive sizes
                         (or times), at the midpoints of the pairs
  power_fit              slope of ln y against ln x (direct fit of Eq. (12))
  stderr                 sigma / sqrt(n - 1) over independent realizations
"""
from __future__ import annotations

import numpy as np


def shape(values):
    """(S, Q) of a sample: Phi_3 / Phi_2^(3/2) and Phi_4 / Phi_2^2 - 3 with
    Phi_n the n-th central moment of the sample."""
    v = np.asarray(values, dtype=np.float64)
    d = v - v.mean()
    p2, p3, p4 = (d ** 2).mean(), (d ** 3).mean(), (d ** 4).mean()
    return float(p3 / p2 ** 1.5), float(p4 / p2 ** 2 - 3.0)


def height_shape(records):
    """(S_h, Q_h) from moment records (dicts with phi2, phi3, phi4): the
    central moments of each state's height distribution averaged over the
    states, then combined as in Eqs. (14)-(15)."""
    p = np.array([[r["phi2"], r["phi3"], r["phi4"]] for r in records], dtype=np.float64)
    p2, p3, p4 = p.mean(axis=0)
    return float(p3 / p2 ** 1.5), float(p4 / p2 ** 2 - 3.0)


def effective_exponent(x, y):
    """Eq. (8): slopes of ln y between consecutive points, placed at the
    midpoints (x_i + x_{i-1}) / 2 of each pair."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    slopes = np.diff(np.log(y)) / np.diff(np.log(x))
    return (x[1:] + x[:-1]) / 2.0, slopes


def power_fit(x, y):
    """Least-squares slope and intercept of ln y against ln x."""
    slope, icept = np.polyfit(np.log(np.asarray(x, dtype=np.float64)),
                              np.log(np.asarray(y, dtype=np.float64)), 1)
    return float(slope), float(icept)


def stderr(values):
    """Standard error over n independent realizations: sigma / sqrt(n - 1)
    (population sigma)."""
    v = np.asarray(values, dtype=np.float64)
    return float(v.std() / np.sqrt(max(v.size - 1, 1)))
