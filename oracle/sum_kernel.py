"""Right-hand side for kernels that depend on the total size only: TEST INFRASTRUCTURE.

For C^(d)_{i_1..i_d} = f(i_1 + ... + i_d) the definitions of Sec. 1 collapse:
in the gain sum every tuple with i_1 + ... + i_d = k carries the same kernel
value f(k), so

    p_k^(d) = f(k) (n^{*d})_k / d!,

with n^{*d} the d-fold linear convolution power of n (sizes as indices); in the
loss sum the tuple (i, k) has kernel value f(s + k), s = i_1 + ... + i_{d-1},
and grouping the tuples by s gives

    q_k^(d) = -n_k / (d-1)! * sum_s f(s + k) (n^{*(d-1)})_s.

This needs no factorisation of the kernel at all, so it measures a compressed
CP kernel's error (compression and evaluation together) against the exact
function, and pins the CP path on function-of-sum kernels.  Convolutions are
direct sums for short supports and numpy FFTs (a library step) otherwise.
"""
from __future__ import annotations

import math

import numpy as np


def _pow2_at_least(x: int) -> int:
    L = 1
    while L < x:
        L *= 2
    return L


def _convolve(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Full linear convolution of two real vectors."""
    if a.size * b.size <= 1 << 24:
        return np.convolve(a, b)
    L = _pow2_at_least(a.size + b.size - 1)
    return np.fft.irfft(np.fft.rfft(a, L) * np.fft.rfft(b, L), L)[: a.size + b.size - 1]


def rhs_sum_kernel(D: int, N: int, fvals: np.ndarray, n: np.ndarray):
    """Returns (p, q) as (D+1, N) arrays, row d = p^(d), q^(d) for k = 1..N.

    fvals[s] = f(s) for s = 0..D*N (fvals[0] and fvals[1] are never used)."""
    fvals = np.asarray(fvals, dtype=np.float64)
    assert fvals.size >= D * N + 1
    n = np.asarray(n, dtype=np.float64)
    nz = np.nonzero(n)[0]
    K = int(nz[-1]) + 1 if nz.size else 0      # n_k = 0 for k > K
    x = np.zeros(K + 1)
    x[1:] = n[:K]                               # x[s] = n_s, sizes as indices
    p = np.zeros((D + 1, N))
    q = np.zeros((D + 1, N))
    if K == 0:
        return p, q
    power = {1: x}
    for d in range(2, D + 1):
        power[d] = _convolve(power[d - 1], x)   # support [d, d K]
        c = power[d]
        m = min(N, c.size - 1)
        p[d, :m] = fvals[1:m + 1] * c[1:m + 1] / math.factorial(d)
        # loss: sum over s of f(s + k) (n^{*(d-1)})_s, for the k with n_k != 0
        prev = power[d - 1]
        S = prev.size - 1                        # s in [0, S]
        if K * (S + 1) <= 1 << 26:
            corr = np.array([np.dot(prev, fvals[k:k + S + 1]) for k in range(1, K + 1)])
        else:
            full = _convolve(prev[::-1].copy(), fvals[: S + K + 1])
            corr = full[S + 1:S + K + 1]
        q[d, :K] = -n[:K] * corr / math.factorial(d - 1)
    return p, q
