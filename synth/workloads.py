"""Synthetic CP kernels and initial data shaped like the paper's workloads.

A kernel of collision order d is given as canonical polyadic (CP) factors
    C^(d)_{i_1..i_d} = sum_r prod_m U^(d)_m(i_m, r)
and is stored here as a float64 array ``U`` of shape ``(d, R_d, N)`` with
``U[m-1, r, i-1] = U^(d)_m(i, r)``.  Mode ``m = d`` is the mode that carries the
size index k in the loss term.  A whole kernel set is a dict ``{d: U}`` for
d = 2..D (a missing d, or R_d = 0, means that collision order is absent).

Every generator is deterministic; random ones take an explicit seed and draw
from numpy's PCG64.
"""
from __future__ import annotations

from itertools import permutations

import numpy as np

__all__ = [
    "sizes", "kernel_constant", "kernel_brownian_sum", "kernel_ballistic",
    "kernel_additive", "kernel_random", "kernel_random_first_mode", "kernel_random_symmetric",
    "kernel_generalized_brownian", "brownian_tt_cores", "n0_monodisperse", "n0_exponential",
    "n0_uniform_head", "n0_random_dense", "CONFIGS", "config", "build_kernel", "build_n0",
    "serving_requests", "sum_kernel_values", "kernel_expsum",
]


def sizes(N: int) -> np.ndarray:
    """Particle sizes 1..N as float64."""
    return np.arange(1, N + 1, dtype=np.float64)


def _ones(N):
    return np.ones(N, dtype=np.float64)


def kernel_constant(D: int, N: int) -> dict:
    """C^(d) == 1 for every d: one rank-1 term whose columns are all exactly 1.0."""
    return {d: np.ones((d, 1, N), dtype=np.float64) for d in range(2, D + 1)}


def kernel_brownian_sum(D: int, N: int, mu: float = 1.0 / 3.0) -> dict:
    """C^(d) = (sum_m i_m^mu)(sum_l i_l^-mu): R_d = d^2 terms indexed by (m, l).

    Mode m carries i^mu and mode l carries i^-mu; when m == l that mode's column
    is the product i^mu * i^-mu written as the exact value 1.0.  Other modes 1.0.
    """
    s = sizes(N)
    up, dn = s ** mu, s ** (-mu)
    out = {}
    for d in range(2, D + 1):
        U = np.ones((d, d * d, N), dtype=np.float64)
        r = 0
        for m in range(d):
            for l in range(d):
                if m != l:
                    U[m, r] = up
                    U[l, r] = dn
                r += 1
        out[d] = U
    return out


def kernel_ballistic(D: int, N: int, a: float = 0.4) -> dict:
    """C^(d) = sum_{m != l} (i_m / i_l)^a: R_d = d(d-1) terms indexed by (m, l)."""
    s = sizes(N)
    up, dn = s ** a, s ** (-a)
    if a == 0.0:
        up = dn = _ones(N)
    out = {}
    for d in range(2, D + 1):
        U = np.ones((d, d * (d - 1), N), dtype=np.float64)
        r = 0
        for m in range(d):
            for l in range(d):
                if m == l:
                    continue
                U[m, r] = up
                U[l, r] = dn
                r += 1
        out[d] = U
    return out


def kernel_additive(D: int, N: int) -> dict:
    """C^(d) = sum_m i_m: R_d = d terms; term r = m has i in mode m, 1.0 elsewhere."""
    s = sizes(N)
    out = {}
    for d in range(2, D + 1):
        U = np.ones((d, d, N), dtype=np.float64)
        for m in range(d):
            U[m, m] = s
        out[d] = U
    return out


def kernel_random(D: int, N: int, ranks, seed: int, low=0.0, high=1.0) -> dict:
    """Non-symmetric random factors U(low, high); ``ranks[d]`` or an int for all d."""
    rng = np.random.default_rng(seed)
    out = {}
    for d in range(2, D + 1):
        R = ranks[d] if isinstance(ranks, dict) else int(ranks)
        out[d] = rng.uniform(low, high, size=(d, R, N))
    return out


def kernel_random_first_mode(D: int, N: int, ranks, seed: int) -> dict:
    """Random U(0,1) first-mode columns, every other mode 1.0 (one column shared
    by every rank-one term of every order)."""
    rng = np.random.default_rng(seed)
    out = {}
    for d in range(2, D + 1):
        R = ranks[d] if isinstance(ranks, dict) else int(ranks)
        U = np.ones((d, R, N), dtype=np.float64)
        U[0] = rng.uniform(0.0, 1.0, size=(R, N))
        out[d] = U
    return out


def kernel_random_symmetric(D: int, N: int, ranks, seed: int) -> dict:
    """Symmetric random kernel: each rank-one term uses one column on every mode."""
    rng = np.random.default_rng(seed)
    out = {}
    for d in range(2, D + 1):
        R = ranks[d] if isinstance(ranks, dict) else int(ranks)
        cols = rng.uniform(0.0, 1.0, size=(R, N))
        out[d] = np.broadcast_to(cols, (d, R, N)).copy()
    return out


def kernel_generalized_brownian(N: int, mus) -> np.ndarray:
    """Factors of the generalized Brownian kernel of Sec. 2, eq. (ch3.eq17).

    C[mu_1..mu_d] = sum over permutations sigma of prod_j i_{sigma(j)}^{mu_j}: one
    rank-one term per permutation, so R = d!.  Returns a (d, d!, N) array.
    """
    d = len(mus)
    s = sizes(N)
    perms = list(permutations(range(d)))
    U = np.ones((d, len(perms), N), dtype=np.float64)
    for r, sig in enumerate(perms):
        for j in range(d):
            U[sig[j], r] = s ** mus[j]
    return U


def sum_kernel_values(smin: int, smax: int, power: float = 0.5) -> np.ndarray:
    """Values f(s) = s**power for the integers s in [smin, smax]: the kernel
    C^(d)(i) = (i_1 + ... + i_d)**power depends on the total size only."""
    return np.arange(smin, smax + 1, dtype=np.float64) ** power


def kernel_expsum(D: int, N: int, alpha, w, weighted: bool = False) -> dict:
    """CP factors of C^(d)(i) = w_0 + sum_r w_r exp(-alpha_r (i_1 + ... + i_d)) for
    every d in [2, D], rank R+1 per order, with E[0] = ones and
    E[r] = exp(-alpha_r i).  Unweighted: term r has w_r E[r] in mode 1 and E[r]
    in the other modes, returned per order as a list of d arrays of shape
    (R+1, N) sharing two arrays.  Weighted: every mode of term r is E[r] and
    the term carries the weight w_r, returned as {"U": [E]*d, "weight": w}."""
    s = sizes(N)
    alpha = np.asarray(alpha, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    E = np.ones((alpha.size + 1, N), dtype=np.float64)
    for r, a in enumerate(alpha):
        E[r + 1] = np.exp(-a * s)
    if weighted:
        return {d: {"U": [E] * d, "weight": w} for d in range(2, D + 1)}
    W = E * w[:, None]
    return {d: [W] + [E] * (d - 1) for d in range(2, D + 1)}


def brownian_tt_cores(N: int, mus) -> list:
    """Tensor-train cores of the generalized Brownian kernel C[mu_1..mu_D] (the
    sum over permutations, Sec. 2) as constructed in the proof of Sec. 2's rank
    theorem: rank index r_lambda <-> a subset of {1..D} of size lambda (subsets
    in lexicographic order), ranks C(D, lambda); core lambda+1 maps subset S to
    S + {xi} with the entry i^mu_xi, and is zero otherwise.  Core m is an array
    of shape (r_{m-1}, N, r_m)."""
    from itertools import combinations
    D = len(mus)
    s = sizes(N)
    subsets = [list(combinations(range(D), lam)) for lam in range(D + 1)]
    index = [{S: k for k, S in enumerate(subs)} for subs in subsets]
    cores = []
    for lam in range(D):                       # core lam+1: subsets of size lam -> lam+1
        H = np.zeros((len(subsets[lam]), N, len(subsets[lam + 1])), dtype=np.float64)
        for a, S in enumerate(subsets[lam]):
            for xi in range(D):
                if xi in S:
                    continue
                b = index[lam + 1][tuple(sorted(S + (xi,)))]
                H[a, :, b] = s ** mus[xi]
        cores.append(H)
    return cores


def n0_monodisperse(N: int) -> np.ndarray:
    n = np.zeros(N, dtype=np.float64)
    n[0] = 1.0
    return n


def n0_exponential(N: int, scale: float = 8.0) -> np.ndarray:
    """n_k(0) = exp(-k/scale) / Z with Z = sum_{k=1}^{N} exp(-k/scale)."""
    v = np.exp(-sizes(N) / scale)
    return v / v.sum()


def n0_uniform_head(N: int, seed: int, kmax: int = 16) -> np.ndarray:
    """Weights w_k ~ U(0,1) (PCG64(seed)) on k in [1, kmax], zero beyond, sum 1."""
    rng = np.random.default_rng(seed)
    n = np.zeros(N, dtype=np.float64)
    k = min(kmax, N)
    w = rng.uniform(0.0, 1.0, size=k)
    n[:k] = w / w.sum()
    return n


def n0_random_dense(N: int, seed: int, decay: float = 0.0) -> np.ndarray:
    """Dense positive state: U(0,1) weights times exp(-decay*k), sum 1."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.0, 1.0, size=N) * np.exp(-decay * sizes(N))
    return w / w.sum()


# The benchmark workloads: kernels, initial data and step sizes.  "prec" names the
# arithmetic of the spectral path; the state itself is always float64.
CONFIGS = {
    "C1": dict(D=3, N=64, kernel=("constant",), n0=("monodisperse",),
               dt=1e-3, t_end=1.0, prec="fp64"),
    "C2": dict(D=3, N=4096, kernel=("brownian_sum", 1.0 / 3.0), n0=("exponential", 8.0),
               dt=1e-3, t_end=10.0, prec="fp64"),
    "C3": dict(D=4, N=65536, kernel=("ballistic", 0.4), n0=("uniform_head", 3, 16),
               dt=5e-4, t_end=0.5, prec="fp32c"),
    # C5a: 10 Heun steps inside explicit Heun's stability interval.  The loss
    # rate of size k under the additive kernel at unit mass is about
    # k (1 + 1 + 1/2 + 1/6) for D = 5, 2.8e6 at k = N = 2^20, so h must stay
    # below 2 / 2.8e6 = 7e-7: at h = 1e-4 the rounding noise of the far tail
    # grows by about 1e4 per step and the state overflows within 10 steps.
    "C5a": dict(D=5, N=1 << 20, kernel=("additive",), n0=("uniform_head_batch", 64, 16),
                dt=5e-7, t_end=5e-6, prec="fp32c"),
}


def build_kernel(D: int, N: int, spec) -> dict:
    kind = spec[0]
    if kind == "constant":
        return kernel_constant(D, N)
    if kind == "brownian_sum":
        return kernel_brownian_sum(D, N, spec[1])
    if kind == "ballistic":
        return kernel_ballistic(D, N, spec[1])
    if kind == "additive":
        return kernel_additive(D, N)
    raise ValueError(f"unknown kernel spec {spec!r}")


def build_n0(N: int, spec) -> np.ndarray:
    kind = spec[0]
    if kind == "monodisperse":
        return n0_monodisperse(N)
    if kind == "exponential":
        return n0_exponential(N, spec[1])
    if kind == "uniform_head":
        return n0_uniform_head(N, spec[1], spec[2])
    raise ValueError(f"unknown initial-data spec {spec!r}")


def config(name: str) -> dict:
    """Materialise a named workload: returns dict(D, N, kernel, n0, dt, t_end, prec)."""
    c = dict(CONFIGS[name])
    c["kernel"] = build_kernel(c["D"], c["N"], c["kernel"])
    if c["n0"][0] == "uniform_head_batch":
        B, kmax = c["n0"][1], c["n0"][2]
        c["n0"] = np.stack([n0_uniform_head(c["N"], s, kmax) for s in range(B)])
    else:
        c["n0"] = build_n0(c["N"], c["n0"])
    c["name"] = name
    return c


def serving_requests(count: int, seed: int = 4, t_end_range=(1.0, 20.0), dt: float = 1e-3,
                     log2n_range=(10, 16), kmax: int = 16, steps_range=None):
    """Solve requests shaped like the serving workload: N = 2^round(U[10,16]),
    D uniform in {2,3,4}, ballistic-like kernel with a ~ U[0, 0.9], initial data
    uniform on [1, kmax] (seeded per request), t_end ~ U[t_end_range].

    With ``steps_range`` the request instead takes a step size inside explicit
    Heun's stability interval, dt = min(dt, 1/(D^2 N^a)) (the loss rate of the
    largest size grows like D^2 N^a for this kernel), and a step count drawn
    from U[steps_range], so t_end = steps * dt."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        N = 1 << int(round(rng.uniform(*log2n_range)))
        D = int(rng.integers(2, 5))
        a = float(rng.uniform(0.0, 0.9))
        t_end = float(rng.uniform(*t_end_range))
        h = dt
        if steps_range is not None:
            h = min(dt, 1.0 / (D * D * float(N) ** a))
            t_end = int(rng.integers(steps_range[0], steps_range[1] + 1)) * h
        out.append(dict(D=D, N=N, a=a, t_end=t_end, dt=h, n0_seed=1000 + i,
                        kernel=kernel_ballistic(D, N, a), n0=n0_uniform_head(N, 1000 + i, kmax)))
    return out
