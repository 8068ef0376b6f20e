"""Tracking horizon (Sec. IV-C): a sequence of one-minute periods whose loads
drift, each period solved warm from the previous period's solution, with the
generators' real power ramp-limited between periods: |p_{t+1} - p_t| <= r_g,
r_g = 2% of the generator's upper limit.

The paper interpolates hourly system demand of a real system into minutes,
with the load changing by up to 5% over 30 minutes. That profile is not
available; `load_profile` stands in for it with a smooth system-wide factor
that rises by `drift` over the horizon (zero slope at both ends, like a
minute-interpolated hourly curve between two hourly points). Every bus load
of period t is the base load times the factor of period t.

Every step of every solve runs in the HIP kernels of libacopf.so; this module
only sequences the periods and computes the ramp-limited bounds on the host.
"""
from __future__ import annotations

import time

import numpy as np

from . import acopf as A
from .gridgen import Grid


def load_profile(periods: int = 30, drift: float = 0.05) -> np.ndarray:
    """System-wide load factor per period: 1 + drift * s(t / (periods - 1)),
    s(x) = 3x^2 - 2x^3 (smooth, monotone, s(0) = 0, s(1) = 1)."""
    if periods < 1:
        raise ValueError("periods must be >= 1")
    x = np.arange(periods) / max(periods - 1, 1)
    return 1.0 + drift * (3.0 * x * x - 2.0 * x * x * x)


def ramp_bounds(pmin: np.ndarray, pmax: np.ndarray, p_prev: np.ndarray, frac: float = 0.02):
    """Bounds for the next period: [max(pmin, p - r), min(pmax, p + r)] with
    r = frac * pmax (Sec. IV-C). p_prev within [pmin, pmax] keeps them non-empty."""
    r = frac * pmax
    p = np.clip(p_prev, pmin, pmax)
    return np.maximum(pmin, p - r), np.minimum(pmax, p + r)


def generator_p(u: np.ndarray, n_gen: int) -> np.ndarray:
    """Real power of each generator from a canonical coupling vector."""
    return np.asarray(u[0:2 * n_gen:2], dtype=np.float64).copy()


def track(solver: A.Solver, grid: Grid, index: int = 0, periods: int = 30,
          drift: float = 0.05, ramp: float = 0.02) -> list[dict]:
    """Solve `periods` periods of grid `index` of `solver`: the first cold, the
    rest warm with ramp-limited generator bounds. Returns one record per
    period (status, inner iterations, seconds, ||c(x)||_inf, objective, and
    max_g |p_t - p_{t-1}| / r_g, which the ramp limits keep <= 1)."""
    factor = load_profile(periods, drift)
    pmin0 = np.asarray(grid.pmin, dtype=np.float64)
    pmax0 = np.asarray(grid.pmax, dtype=np.float64)
    out = []
    p_prev = None
    for t in range(periods):
        if t == 0:
            solver.update_gen_bounds(index, pmin0, pmax0)
        else:
            lo, hi = ramp_bounds(pmin0, pmax0, p_prev, ramp)
            solver.update_gen_bounds(index, lo, hi)
        solver.update_loads(index, grid.pd * factor[t], grid.qd * factor[t])
        t0 = time.perf_counter()
        if t == 0:
            solver.start(index, A.COLD)
        else:
            solver.start(index, A.WARM)
        while solver.is_running(index):
            solver.run(1 << 20)
        seconds = time.perf_counter() - t0
        _, res = solver.poll(index)
        p = generator_p(solver.get("u", index), grid.n_gen)
        ratio = 0.0
        if p_prev is not None and p.size:
            r = ramp * pmax0
            ratio = float(np.max(np.abs(p - p_prev)[r > 0] / r[r > 0], initial=0.0))
        q = solver.quality(index)
        out.append({"period": t, "load_factor": float(factor[t]), "status": res["status"],
                    "inner_iters": res["inner_iters"], "seconds": seconds,
                    "max_violation": q["max_violation"], "objective": res["objective"],
                    "ramp_ratio": ratio})
        p_prev = p
    return out
