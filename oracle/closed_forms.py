"""Closed forms that pin the oracle (test infrastructure only).

Constant kernel C^(d) == 1: summing the operators of Sec. 1 over k (no mass
lost past N) gives dM0/dt = sum_d [M0^d/d! - M0^d/(d-1)!] = -sum_d (d-1) M0^d/d!.
For D = 3 (d = 2 and 3) with M0(0) = 1, separating variables gives
    t = 2/M - 2 + (4/3) ln(5M / (3 + 2M)).
Binary constant kernel (D = 2, the binary equation of Sec. 1 with the usual 1/2),
monodisperse start: n_k(t) = M^2 (1 - M)^(k-1) with M = 2/(2 + t).
"""
from __future__ import annotations

import math

import numpy as np

from .heun import time_grid


def m0_rhs_constant_kernel(M: float, D: int) -> float:
    return -sum((d - 1) * M ** d / math.factorial(d) for d in range(2, D + 1))


def m0_constant_kernel_d3(t: float) -> float:
    """Invert t(M) = 2/M - 2 + (4/3) ln(5M/(3+2M)) on (0, 1] by bisection."""
    def t_of(M):
        return 2.0 / M - 2.0 + (4.0 / 3.0) * math.log(5.0 * M / (3.0 + 2.0 * M))
    lo, hi = 1e-12, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if t_of(mid) > t:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def scalar_heun(g, y0: float, dt: float, t_end: float) -> float:
    y = float(y0)
    for h in time_grid(dt, t_end):
        k1 = g(y)
        k2 = g(y + h * k1)
        y = y + 0.5 * h * (k1 + k2)
    return y


def binary_constant_monodisperse(N: int, t: float) -> np.ndarray:
    M = 2.0 / (2.0 + t)
    k = np.arange(1, N + 1, dtype=np.float64)
    return M * M * (1.0 - M) ** (k - 1)
