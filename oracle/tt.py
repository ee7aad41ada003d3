"""Kernels in tensor-train form (TEST INFRASTRUCTURE: oracle side).

The paper writes a kernel tensor of order d in TT form (Sec. 2, eq. (ch3.eq4)):

    C_{i_1..i_d} = sum_{r_1..r_{d-1}} H^(1)_{1, i_1, r_1} H^(2)_{r_1, i_2, r_2} ... H^(d)_{r_{d-1}, i_d, 1},

a core H^(m) being an array of shape (r_{m-1}, N, r_m) with r_0 = r_d = 1.

* ``tt_full``   the dense tensor C from its cores (the contraction written out,
                one matrix product per mode, at every index tuple; tiny N only)
* ``tt_paths``  the same kernel as CP factors: one rank-one term per rank path
                (r_1, .., r_{d-1}), mode m's column being H^(m)_{r_{m-1}, :, r_m};
                the sum over paths IS the TT sum, term by term
* ``rhs_dense`` the right-hand side of Sec. 1 from dense kernel tensors: the
                literal sums p_k^(d) and q_k^(d) over index tuples (tiny N only)

None of this shares code with the library: the library never expands rank
paths for a TT plan and evaluates the chain of core matrices per frequency bin.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def tt_full(cores) -> np.ndarray:
    """Dense C of shape (N,)*d from cores (r_{m-1}, N, r_m)."""
    d = len(cores)
    N = cores[0].shape[1]
    C = np.zeros((N,) * d)
    for idx in itertools.product(range(N), repeat=d):
        v = np.ones((1, 1))
        for m in range(d):
            v = v @ cores[m][:, idx[m], :]
        C[idx] = v[0, 0]
    return C


def tt_paths(cores) -> np.ndarray:
    """CP factors (d, P, N) with P = prod r_1..r_{d-1}: path (r_1, .., r_{d-1}) in
    lexicographic order, U[m-1, p] = H^(m)[r_{m-1}, :, r_m]."""
    d = len(cores)
    N = cores[0].shape[1]
    inner = [cores[m].shape[2] for m in range(d - 1)]
    paths = list(itertools.product(*[range(r) for r in inner]))
    U = np.zeros((d, len(paths), N))
    for p, path in enumerate(paths):
        full = (0,) + path + (0,)
        for m in range(d):
            U[m, p] = cores[m][full[m], :, full[m + 1]]
    return U


def rhs_dense(D: int, N: int, dense: dict, n: np.ndarray):
    """(p, q) arrays of shape (N,) from dense kernels {d: C of shape (N,)*d}:

        p_k^(d) =  1/d!       sum_{|i| = k} C_i n_{i_1} .. n_{i_d}
        q_k^(d) = -n_k/(d-1)! sum_{i in [1,N]^(d-1)} C_{(i,k)} n_{i_1} .. n_{i_{d-1}}

    (Sec. 1; index k in the last mode), summed over d."""
    n = np.asarray(n, dtype=np.float64)
    p = np.zeros(N)
    q = np.zeros(N)
    for d, C in dense.items():
        for idx in itertools.product(range(N), repeat=d):
            w = C[idx] * math.prod(n[i] for i in idx)
            s = sum(idx) + d          # total size (indices are size - 1)
            if s <= N:
                p[s - 1] += w / math.factorial(d)
        for idx in itertools.product(range(N), repeat=d - 1):
            w = math.prod(n[i] for i in idx)
            for k in range(N):
                q[k] -= n[k] * C[idx + (k,)] * w / math.factorial(d - 1)
    return p, q
