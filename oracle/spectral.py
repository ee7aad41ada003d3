"""CP-FFT evaluation of the right-hand side with numpy's FFT as a library step.

Sec. 1 (CP remark): with C^(d) in CP form every rank-one term of the gain sum is
a d-fold linear convolution of the weighted vectors x_{m,r}[i] = U_m(i, r) n_i,
and every term of the loss sum is a product of dot products.  This module
writes that out directly: one real FFT per (d, m, r), a product of spectra per
(d, r), one inverse per d, at a length Lo >= d*N + 1 so that no cyclic wrap can
occur at all.  No column sharing, no fusion.  Test infrastructure only.
"""
from __future__ import annotations

import math

import numpy as np


def _pow2_at_least(x: int) -> int:
    L = 1
    while L < x:
        L *= 2
    return L


def rhs_fft(D: int, N: int, kernel: dict, n: np.ndarray):
    """Returns (p, q) as (D+1, N) float64 arrays, row d = p^(d), q^(d) for k = 1..N."""
    n = np.asarray(n, dtype=np.float64)
    p = np.zeros((D + 1, N))
    q = np.zeros((D + 1, N))
    for d in range(2, D + 1):
        U = kernel.get(d)
        if U is None or U.shape[1] == 0:
            continue
        R = U.shape[1]
        Lo = _pow2_at_least(d * N + 1)
        spec = np.zeros(Lo // 2 + 1, dtype=np.complex128)
        for r in range(R):
            prod = np.ones(Lo // 2 + 1, dtype=np.complex128)
            for m in range(d):
                x = np.zeros(Lo)
                x[1:N + 1] = U[m, r] * n          # index = particle size
                prod = prod * np.fft.rfft(x)
            spec += prod
        y = np.fft.irfft(spec, Lo)
        p[d] = y[1:N + 1] / math.factorial(d)
        for r in range(R):
            dots = 1.0
            for m in range(d - 1):
                dots *= float(np.dot(U[m, r], n))
            q[d] -= n * U[d - 1, r] * dots / math.factorial(d - 1)
    return p, q


def total_rhs(p: np.ndarray, q: np.ndarray) -> np.ndarray:
    """f_k = sum_d (p_k^(d) + q_k^(d)) (Sec. 1, the multi-particle system)."""
    return p.sum(axis=0) + q.sum(axis=0)
