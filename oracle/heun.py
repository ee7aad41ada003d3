"""Explicit second-order Runge-Kutta in Heun's form (Sec. 3: two right-hand-side
evaluations per step).  Test infrastructure only.

Time grid (a reading; the paper does not state one): with h the requested step,
the number of steps is round(t_end/h) when t_end/h is within 1e-9 (relative) of
an integer, else ceil(t_end/h), and then the last step is shortened to
t_end - (nsteps-1)*h.  Step j starts at j*h, never at an accumulated sum.
"""
from __future__ import annotations

import math

import numpy as np


def time_grid(dt: float, t_end: float):
    """List of step sizes covering [0, t_end]."""
    if t_end == 0.0:
        return []
    ratio = t_end / dt
    near = round(ratio)
    if near >= 1 and abs(ratio - near) <= 1e-9 * ratio:
        return [dt] * int(near)
    ns = int(math.ceil(ratio))
    return [dt] * (ns - 1) + [t_end - (ns - 1) * dt]


def heun_solve(rhs, n0: np.ndarray, dt: float, t_end: float, callback=None):
    """n_{j+1} = n_j + h/2 (f(n_j) + f(n_j + h f(n_j)))."""
    n = np.array(n0, dtype=np.float64, copy=True)
    for j, h in enumerate(time_grid(dt, t_end)):
        k1 = rhs(n)
        k2 = rhs(n + h * k1)
        n = n + 0.5 * h * (k1 + k2)
        if callback is not None:
            callback(j, n)
    return n
