"""Host-side analysis of measured runs: surface tension from the Laplace law and the power law of
droplet spreading (Sec. III.B). Plain least squares on numbers the GPU produced."""
from __future__ import annotations

import math

import numpy as np


def laplace_gamma(radii, dp) -> tuple[float, float]:
    """Surface tension from the 2D Laplace law dp = gamma / R (+ intercept): least squares of the
    pressure jumps dp against 1/R. Returns (gamma, intercept)."""
    x = 1.0 / np.asarray(radii, dtype=np.float64)
    A = np.column_stack([x, np.ones_like(x)])
    (g, c), *_ = np.linalg.lstsq(A, np.asarray(dp, dtype=np.float64), rcond=None)
    return float(g), float(c)


def inertial_time(rho: float, radius: float, gamma: float) -> float:
    """tau_rho = sqrt(rho R^3 / gamma), the inertial time of the spreading law."""
    return math.sqrt(rho * radius ** 3 / gamma)


def fit_power_law(t, r, t_lo: float, t_hi: float) -> tuple[float, float, int]:
    """Least squares of log r = log C + n log t over samples with t_lo <= t <= t_hi and r > 0.
    Returns (C, n, samples used)."""
    t = np.asarray(t, dtype=np.float64)
    r = np.asarray(r, dtype=np.float64)
    sel = (t >= t_lo) & (t <= t_hi) & np.isfinite(r) & (r > 0)
    if sel.sum() < 2:
        return float("nan"), float("nan"), int(sel.sum())
    A = np.column_stack([np.log(t[sel]), np.ones(int(sel.sum()))])
    (n, lc), *_ = np.linalg.lstsq(A, np.log(r[sel]), rcond=None)
    return float(math.exp(lc)), float(n), int(sel.sum())
