"""Pins for the oracle (CPU only).  Each check ties the oracle to something other
than itself: hand-derived values from the operator definitions of Sec. 1, the
binary equation of Sec. 1 written with a dense kernel matrix, moment identities
that follow from the definitions, closed-form solutions, and agreement of three
independently written evaluations (literal sums, per-rank direct convolutions,
per-rank FFT products)."""
import math

import numpy as np
import pytest

import oracle
import synth
from conftest import read_golden_kv, read_golden_table


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


ALL_RHS = [("direct", oracle.rhs_direct), ("conv", oracle.rhs_conv), ("fft", oracle.rhs_fft)]


@pytest.mark.parametrize("name,fn", ALL_RHS)
def test_golden_binary_hand(name, fn):
    rows = np.array(read_golden_table("binary_rank1_N3.txt"))
    kern = {2: np.array([[[1.0, 2.0, 3.0]], [[1.0, 10.0, 100.0]]])}
    n = np.array([1.0, 0.5, 0.25])
    p, q = fn(2, 3, kern, n)
    assert np.allclose(p[2], rows[:, 1], rtol=0, atol=1e-13)
    assert np.allclose(q[2], rows[:, 2], rtol=0, atol=1e-13)
    assert np.allclose(oracle.total_rhs(p, q), rows[:, 3], rtol=0, atol=1e-13)


@pytest.mark.parametrize("name,fn", ALL_RHS)
def test_golden_ternary_hand(name, fn):
    rows = np.array(read_golden_table("ternary_rank1_N4.txt"))
    kern = {3: np.array([[[1.0, 2.0, 0.0, 0.0]], [[3.0, 1.0, 0.0, 0.0]], [[1.0, 5.0, 7.0, 2.0]]])}
    n = np.array([1.0, 2.0, 0.5, 1.0])
    p, q = fn(3, 4, kern, n)
    assert np.all(p[2] == 0) and np.all(q[2] == 0)
    assert np.allclose(p[3], rows[:, 1], rtol=0, atol=1e-12)
    assert np.allclose(q[3], rows[:, 2], rtol=0, atol=1e-12)
    assert np.allclose(oracle.total_rhs(p, q), rows[:, 3], rtol=0, atol=1e-12)


@pytest.mark.parametrize("D,N,R,seed", [(2, 17, 3, 1), (3, 13, 2, 2), (4, 9, 2, 3), (5, 7, 2, 4), (3, 24, 4, 5)])
def test_three_evaluations_agree(D, N, R, seed):
    kern = synth.kernel_random(D, N, R, seed)
    n = synth.n0_random_dense(N, seed + 100)
    pd, qd = oracle.rhs_direct(D, N, kern, n)
    pc, qc = oracle.rhs_conv(D, N, kern, n)
    pf, qf = oracle.rhs_fft(D, N, kern, n)
    for d in range(2, D + 1):
        scale = max(np.abs(pd[d]).max(), np.abs(qd[d]).max())
        assert np.abs(pd[d] - pc[d]).max() <= 1e-14 * scale
        assert np.abs(qd[d] - qc[d]).max() <= 1e-14 * scale
        assert np.abs(pd[d] - pf[d]).max() <= 1e-13 * scale
        assert np.abs(qd[d] - qf[d]).max() <= 1e-14 * scale


def test_binary_case_is_the_dense_binary_equation():
    """D = 2 reduces to the binary equation of Sec. 1 (with the loss sum over n_i):
    dn_k/dt = 1/2 sum_{i+j=k} C_ij n_i n_j - n_k sum_i C_{k,i} n_i, here with the
    dense matrix C = U1 U2^T, so C_{k,i} = C[i, k] (k sits in the second mode)."""
    N = 40
    kern = synth.kernel_random(2, N, 3, 11)
    n = synth.n0_random_dense(N, 12)
    C = kern[2][0].T @ kern[2][1]          # C[i-1, j-1] = sum_r U1(i,r) U2(j,r)
    gain = np.zeros(N)
    for k in range(2, N + 1):
        i = np.arange(1, k)
        gain[k - 1] = 0.5 * np.sum(C[i - 1, k - i - 1] * n[i - 1] * n[k - i - 1])
    loss = -n * (C.T @ n)
    p, q = oracle.rhs_direct(2, N, kern, n)
    assert _rel(p[2], gain) < 1e-14
    assert _rel(q[2], loss) < 1e-14


@pytest.mark.parametrize("fn", [oracle.rhs_direct, oracle.rhs_conv, oracle.rhs_fft])
def test_sum_identities(fn):
    """Summing the definitions over k: if n vanishes beyond N/D, no gain tuple is
    cut by the truncation and sum_k p^(d) = 1/d! sum_r prod_m (U_m[:,r].n), while
    the loss sum always covers all of [1,N]^d: sum_k q^(d) = -1/(d-1)! * the same."""
    D, N = 4, 24
    kern = synth.kernel_random(D, N, 3, 21)
    n = synth.n0_random_dense(N, 22)
    n[N // D:] = 0.0
    p, q = fn(D, N, kern, n)
    for d in range(2, D + 1):
        U = kern[d]
        s = sum(np.prod([U[m, r] @ n for m in range(d)]) for r in range(U.shape[1]))
        assert abs(p[d].sum() - s / math.factorial(d)) <= 1e-14 * s
        assert abs(q[d].sum() + s / math.factorial(d - 1)) <= 1e-14 * s


def test_mass_is_conserved_for_symmetric_kernels():
    """For a symmetric kernel each d-particle collision moves mass from the d
    colliders into one particle of the summed size: sum_k k f_k = 0 while no
    product can exceed size N."""
    D, N = 4, 32
    kern = synth.kernel_random_symmetric(D, N, 2, 31)
    n = synth.n0_random_dense(N, 32)
    n[N // D:] = 0.0
    p, q = oracle.rhs_direct(D, N, kern, n)
    k = np.arange(1, N + 1)
    for d in range(2, D + 1):
        scale = np.sum(k * (np.abs(p[d]) + np.abs(q[d])))
        assert abs(np.sum(k * (p[d] + q[d]))) <= 1e-14 * scale
    # and a non-symmetric kernel breaks it (guards against a vacuous check)
    kn = synth.kernel_random(D, N, 2, 33)
    p2, q2 = oracle.rhs_direct(D, N, kn, n)
    assert abs(np.sum(k * (p2[3] + q2[3]))) > 1e-6 * np.sum(k * np.abs(q2[3]))


def test_constant_kernel_zeroth_moment_rhs():
    D, N = 5, 40
    kern = synth.kernel_constant(D, N)
    n = synth.n0_random_dense(N, 41)
    n[N // D:] = 0.0
    n *= 1.7
    p, q = oracle.rhs_conv(D, N, kern, n)
    M = n.sum()
    assert abs(oracle.total_rhs(p, q).sum() - oracle.m0_rhs_constant_kernel(M, D)) <= 1e-14 * M ** D * 10


def test_constant_kernel_m0_closed_form_trajectory():
    """Config C1 (D=3, N=64, constant kernel, monodisperse, Heun h=1e-3 to t=1)."""
    g = read_golden_kv("constant_kernel_m0.txt")
    assert abs(oracle.m0_constant_kernel_d3(1.0) - g["m0_exact"]) < 1e-15
    c = synth.config("C1")
    D, N = c["D"], c["N"]
    rhs = lambda v: oracle.total_rhs(*oracle.rhs_fft(D, N, c["kernel"], v))
    nT = oracle.heun_solve(rhs, c["n0"], c["dt"], c["t_end"])
    m0 = nT.sum()
    sh = oracle.scalar_heun(lambda M: oracle.m0_rhs_constant_kernel(M, D), 1.0, c["dt"], c["t_end"])
    assert abs(sh - g["m0_scalar_heun_dt1e-3"]) < 1e-15
    assert abs(m0 - sh) < 1e-13
    assert abs(m0 - g["m0_exact"]) < 1e-7          # O(h^2) global error
    # mass is conserved while the tail stays far below N
    assert abs(np.sum(np.arange(1, N + 1) * nT) - 1.0) < 1e-13


def test_binary_constant_kernel_closed_form():
    N, dt, T = 200, 1e-3, 1.0
    kern = synth.kernel_constant(2, N)
    rhs = lambda v: oracle.total_rhs(*oracle.rhs_fft(2, N, kern, v))
    nT = oracle.heun_solve(rhs, synth.n0_monodisperse(N), dt, T)
    exact = oracle.binary_constant_monodisperse(N, T)
    assert np.max(np.abs(nT - exact)) < 1e-7
    assert np.max(np.abs(nT - exact)) > 1e-12      # it is a second-order method, not exact


def test_time_grid():
    assert oracle.time_grid(1e-3, 1.0) == [1e-3] * 1000
    assert oracle.time_grid(0.3, 1.0)[-1] == pytest.approx(0.1)
    assert len(oracle.time_grid(0.3, 1.0)) == 4
    assert oracle.time_grid(0.5, 0.0) == []
    assert len(oracle.time_grid(5e-4, 0.5)) == 1000


def test_sampled_gain_prefix_matches_full():
    """The kmax-limited convolution (used for sampled outputs at large N) agrees
    with the full evaluation on the prefix it computes."""
    D, N = 3, 300
    kern = synth.kernel_ballistic(D, N, 0.4)
    n = synth.n0_random_dense(N, 51, decay=0.01)
    pf, qf = oracle.rhs_conv(D, N, kern, n)
    ps, qs = oracle.rhs_conv(D, N, kern, n, kmax=57)
    assert np.array_equal(ps[:, :57], pf[:, :57])
    assert np.all(np.isnan(ps[2:, 57:]))
    assert np.array_equal(qs, qf)


# ---- planted mistakes: each must be caught by one of the pins above ----------

def _mutant_fft(mutation):
    def rhs(D, N, kernel, n):
        p, q = oracle.rhs_fft(D, N, kernel, n)
        if mutation == "loss_factorial":          # d! instead of (d-1)!
            for d in range(2, D + 1):
                q[d] /= d
        elif mutation == "kmode_first":           # k taken in mode 1
            q = np.zeros_like(q)
            for d in range(2, D + 1):
                U = kernel.get(d)
                if U is None:
                    continue
                for r in range(U.shape[1]):
                    dots = np.prod([U[m, r] @ n for m in range(1, d)])
                    q[d] -= n * U[0, r] * dots / math.factorial(d - 1)
        elif mutation == "drop_last_rank":
            kk = {d: U[:, :-1] for d, U in kernel.items()}
            p, q = oracle.rhs_fft(D, N, kk, n)
        return p, q
    return rhs


@pytest.mark.parametrize("mutation", ["loss_factorial", "kmode_first", "drop_last_rank"])
def test_planted_mistakes_are_caught(mutation):
    fn = _mutant_fft(mutation)
    rows = np.array(read_golden_table("ternary_rank1_N4.txt"))
    kern3 = {3: np.array([[[1.0, 2.0, 0.0, 0.0]], [[3.0, 1.0, 0.0, 0.0]], [[1.0, 5.0, 7.0, 2.0]]])}
    n4 = np.array([1.0, 2.0, 0.5, 1.0])
    caught = False
    p, q = fn(3, 4, kern3, n4)
    caught |= not np.allclose(oracle.total_rhs(p, q), rows[:, 3], rtol=0, atol=1e-12)
    D, N = 4, 9
    kern = synth.kernel_random(D, N, 2, 3)
    n = synth.n0_random_dense(N, 103)
    pd, qd = oracle.rhs_direct(D, N, kern, n)
    pm, qm = fn(D, N, kern, n)
    caught |= _rel(oracle.total_rhs(pm, qm), oracle.total_rhs(pd, qd)) > 1e-10
    assert caught


def test_heun_step_is_heun_not_midpoint():
    """One step of y' = y^2 from y = 1 with h = 0.1, worked by hand: Heun gives
    1 + 0.05 (1 + 1.1^2) = 1.1105 (explicit midpoint would give 1.11025, Euler
    1.1); every two-stage second-order method agrees on linear problems, so a
    nonlinear one pins the stages.  The GPU path's Heun stages are checked
    against this oracle."""
    y = oracle.heun_solve(lambda v: v * v, np.array([1.0]), 0.1, 0.1)
    assert abs(y[0] - 1.1105) < 1e-15
    y2 = oracle.heun_solve(lambda v: v * v, np.array([1.0]), 0.1, 0.2)
    y1 = 1.1105
    assert abs(y2[0] - (y1 + 0.05 * (y1 ** 2 + (y1 + 0.1 * y1 ** 2) ** 2))) < 1e-15


def _brute_sum_kernel(D, N, f, n):
    """Literal sums of Sec. 1 with the dense kernel C_i = f(i_1 + ... + i_d)."""
    import itertools
    p = np.zeros((D + 1, N))
    q = np.zeros((D + 1, N))
    for d in range(2, D + 1):
        for idx in itertools.product(range(1, N + 1), repeat=d):
            s = sum(idx)
            prod = math.prod(n[i - 1] for i in idx)
            c = f(s)
            if s <= N:
                p[d, s - 1] += c * prod / math.factorial(d)
            k = idx[-1]
            q[d, k - 1] -= c * prod / math.factorial(d - 1)
    return p, q


@pytest.mark.parametrize("D,N,seed", [(2, 11, 1), (3, 8, 2), (4, 6, 3), (5, 5, 4)])
def test_sum_kernel_identity_matches_brute_force(D, N, seed):
    """p^(d) = f(k) (n^{*d})_k / d! and the grouped loss sum, against the literal
    sums with a dense kernel tensor (no CP form involved)."""
    f = lambda s: math.sqrt(s) + 0.25 * (s % 3)
    n = synth.n0_random_dense(N, seed)
    fv = np.array([f(s) if s > 0 else 0.0 for s in range(D * N + 1)])
    pb, qb = _brute_sum_kernel(D, N, f, n)
    ps, qs = oracle.rhs_sum_kernel(D, N, fv, n)
    for d in range(2, D + 1):
        scale = max(np.abs(pb[d]).max(), np.abs(qb[d]).max())
        assert np.abs(ps[d] - pb[d]).max() <= 1e-14 * scale
        assert np.abs(qs[d] - qb[d]).max() <= 1e-14 * scale


@pytest.mark.parametrize("D,N", [(3, 9), (5, 6)])
def test_expsum_factors_give_the_sum_kernel(D, N):
    """The CP factors of an exponential sum (synth.kernel_expsum) reproduce the
    function of the total size: the literal CP sums equal the identity."""
    alpha, w = np.array([0.05, 0.4, 1.3]), np.array([0.7, 2.0, -1.5, 0.25])
    kern = {d: np.asarray(v) for d, v in synth.kernel_expsum(D, N, alpha, w).items()}
    fv = np.array([w[0] + np.sum(w[1:] * np.exp(-alpha * s)) for s in range(D * N + 1)])
    n = synth.n0_random_dense(N, 11)
    pd, qd = oracle.rhs_direct(D, N, kern, n)
    ps, qs = oracle.rhs_sum_kernel(D, N, fv, n)
    for d in range(2, D + 1):
        scale = max(np.abs(pd[d]).max(), np.abs(qd[d]).max())
        assert np.abs(ps[d] - pd[d]).max() <= 1e-13 * scale
        assert np.abs(qs[d] - qd[d]).max() <= 1e-13 * scale


def test_sum_kernel_fft_branch_matches_direct_branch():
    """The FFT branches of the identity (dense state) against direct sums: the
    gain prefix against the short-support branch (outputs k < m only involve
    sizes < m), and the loss sum through the identity
    sum_k q_k^(d) = -1/(d-1)! sum_s f(s) (n^{*d})_s with np.convolve powers."""
    D, N = 4, 6000
    n = synth.n0_random_dense(N, 5, decay=1e-3)
    fv = np.sqrt(np.arange(D * N + 1, dtype=np.float64))
    p, q = oracle.rhs_sum_kernel(D, N, fv, n)
    m = 40
    ns = n.copy()
    ns[m:] = 0.0
    ps, qs = oracle.rhs_sum_kernel(D, N, fv, ns)
    x = np.concatenate([[0.0], n])
    power = x
    for d in range(2, D + 1):
        assert np.abs(p[d, :m] - ps[d, :m]).max() <= 1e-13 * np.abs(p[d]).max()
        power = np.convolve(power, x)
        expect = -np.dot(fv[:power.size], power) / math.factorial(d - 1)
        assert abs(q[d].sum() - expect) <= 1e-12 * abs(expect)


@pytest.mark.parametrize("D,N,kf,seed", [
    (2, 50, lambda D, N: synth.kernel_random(D, N, 3, 61), 62),
    (3, 37, lambda D, N: synth.kernel_random(D, N, 2, 63), 64),
    (4, 21, lambda D, N: synth.kernel_ballistic(D, N, 0.4), 65),
    (5, 13, lambda D, N: synth.kernel_additive(D, N), 66),
    (3, 1, lambda D, N: synth.kernel_random(D, N, 2, 67), 68),
])
def test_factored_cpu_version_equals_literal_sums(D, N, kf, seed):
    """The factored CPU evaluation (own FFT, OpenMP) against the literal sums."""
    k = kf(D, N)
    n = synth.n0_random_dense(N, seed)
    ref = oracle.total_rhs(*oracle.rhs_direct(D, N, k, n))
    f, threads = oracle.rhs_factored(D, N, k, n)
    assert threads >= 1
    assert np.max(np.abs(f - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_factored_cpu_version_equals_direct_convolutions():
    """At a size where the literal sums are out of reach: against the per-rank
    direct convolutions, on a dense state (ballistic D=4 kernel, N=3000)."""
    D, N = 4, 3000
    k = synth.kernel_ballistic(D, N, 0.4)
    n = synth.n0_random_dense(N, 69, decay=1e-3)
    ref = oracle.total_rhs(*oracle.rhs_conv(D, N, k, n))
    f, _ = oracle.rhs_factored(D, N, k, n)
    assert np.max(np.abs(f - ref)) <= 1e-12 * np.max(np.abs(ref))
