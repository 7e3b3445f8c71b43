"""Steady-state test of a flow from its mean velocity, sampled every K steps.

A run is steady when its mean velocity U stops changing.  Two situations
look alike to a test of one window's change and are told apart here:

  * converged: the change of U over each of the last `windows` windows is
    below `tol` of U.  One small window is not enough: U of a porous flow
    driven from rest overshoots once, and at the turning point one window
    can change U by almost nothing;
  * noise floor (stagnated): with reduced-precision storage the rounding of
    every stored value leaves U fluctuating from window to window by more
    than `tol`, around a level that no longer moves.  Recognised when, over
    the last `trend_windows` windows, the least-squares trend of U is below
    `tol` of U per window while the window changes flip sign at least
    `min_flips` times (an approach to steady state keeps one sign, apart
    from the single overshoot).

Either way the state is steady to the resolution the storage allows; the
status says which, and `noise` gives the size of the fluctuation.  A
non-finite U means the solve diverged.
"""
from __future__ import annotations

import math

import numpy as np

RUNNING, CONVERGED, NOISE_FLOOR, DIVERGED = "running", "converged", "noise_floor", "diverged"


class SteadyMonitor:
    def __init__(self, tol: float, windows: int = 3, trend_windows: int = 10, min_flips: int = 3):
        if windows < 1 or trend_windows < 2 or min_flips < 1:
            raise ValueError("windows >= 1, trend_windows >= 2 and min_flips >= 1 are required")
        self.tol = float(tol)
        self.windows = int(windows)
        self.trend_windows = int(trend_windows)
        self.min_flips = int(min_flips)
        self.history: list[float] = []
        self.status = RUNNING
        self.trend = float("nan")   # |least-squares slope| / |U| per window over the trend span
        self.noise = float("nan")   # RMS window change / |U| over the trend span

    @property
    def last_change(self) -> float:
        """Relative change of U over the last window (nan before two samples)."""
        h = self.history
        if len(h) < 2 or h[-1] == 0.0:
            return float("nan")
        return abs(h[-1] - h[-2]) / abs(h[-1])

    def push(self, u: float) -> str:
        """Adds the mean velocity after one more window; returns the status."""
        u = float(u)
        self.history.append(u)
        if not math.isfinite(u):
            self.status = DIVERGED
            return self.status
        h = self.history
        scale = abs(h[-1])
        if scale == 0.0:
            return self.status
        w = self.windows
        if len(h) > w and all(abs(h[-j] - h[-j - 1]) < self.tol * scale for j in range(1, w + 1)):
            self.status = CONVERGED
            return self.status
        t = self.trend_windows
        if len(h) > t:
            y = np.asarray(h[-(t + 1):], dtype=np.float64)
            x = np.arange(t + 1, dtype=np.float64)
            x -= x.mean()
            slope = float(np.dot(x, y - y.mean()) / np.dot(x, x))
            d = np.diff(y)
            flips = int(np.count_nonzero(np.sign(d[1:]) * np.sign(d[:-1]) < 0))
            self.trend = abs(slope) / scale
            self.noise = float(np.sqrt(np.mean(d * d))) / scale
            if self.trend < self.tol and flips >= self.min_flips:
                self.status = NOISE_FLOOR
        return self.status

    @property
    def steady(self) -> bool:
        return self.status in (CONVERGED, NOISE_FLOOR)
