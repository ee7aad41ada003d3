"""Tensor-train kernels on the host (no GPU): the generalized Brownian cores
built as in the proof of Sec. 2's rank theorem reproduce the kernel's
definition (the sum over permutations) with ranks C(D, lambda); the library's
expansion of TT cores into rank-one paths reproduces the contraction of the
cores; the planner merges the d! paths of a Brownian kernel into one gain term."""
import itertools
import math

import numpy as np
import pytest

import synth

agg = pytest.importorskip("paper_1905_09071_amd")


def contract(cores, N):
    D = len(cores)
    C = np.zeros((N,) * D)
    for idx in itertools.product(range(N), repeat=D):
        v = np.ones((1, 1))
        for m in range(D):
            v = v @ cores[m][:, idx[m], :]
        C[idx] = v[0, 0]
    return C


def dense_from_cp(U, N):
    D = U.shape[0]
    C = np.zeros((N,) * D)
    for idx in itertools.product(range(N), repeat=D):
        C[idx] = sum(np.prod([U[m, p, idx[m]] for m in range(D)]) for p in range(U.shape[1]))
    return C


@pytest.mark.parametrize("mus", [[0.5, -0.5], [1 / 3, -1 / 3, 0.0], [0.3, -0.3, 0.1, 0.0],
                                 [0.2, -0.1, 0.4, -0.3, 0.0]])
def test_brownian_tt_cores_reproduce_the_definition(mus):
    D, N = len(mus), 5 if len(mus) < 5 else 4
    cores = synth.brownian_tt_cores(N, mus)
    assert [c.shape[2] for c in cores] == [math.comb(D, lam) for lam in range(1, D + 1)]
    s = np.arange(1, N + 1, dtype=np.float64)
    ref = np.zeros((N,) * D)
    for idx in itertools.product(range(N), repeat=D):
        ref[idx] = sum(math.prod(s[idx[sg[j]]] ** mus[j] for j in range(D))
                       for sg in itertools.permutations(range(D)))
    assert np.abs(contract(cores, N) - ref).max() <= 1e-14 * np.abs(ref).max()
    # and the CP form with one rank-one term per permutation (synth's other builder)
    assert np.abs(dense_from_cp(synth.kernel_generalized_brownian(N, mus), N) - ref).max() <= 1e-14 * ref.max()


def test_tt_expand_reproduces_the_contraction():
    """Dense random cores with some all-zero core columns: the expansion keeps
    exactly the paths through non-zero columns and reproduces the tensor."""
    rng = np.random.default_rng(3)
    N, ranks = 6, [1, 2, 3, 1]
    cores = [rng.uniform(-1, 1, size=(ranks[m], N, ranks[m + 1])) for m in range(3)]
    cores[1][0, :, 2] = 0.0
    cores[1][1, :, 0] = 0.0
    U = agg.tt_expand(N, cores)
    paths = [(a, b) for a in range(2) for b in range(3) if np.any(cores[1][a, :, b])]
    assert U.shape == (3, len(paths), N)
    assert np.abs(dense_from_cp(U, N) - contract(cores, N)).max() <= 1e-15 * np.abs(contract(cores, N)).max()


@pytest.mark.parametrize("mus", [[1 / 3, -1 / 3, 0.0], [0.3, -0.3, 0.1, 0.0]])
def test_brownian_tt_plan_merges_the_paths(mus):
    D, N = len(mus), 64
    U = agg.tt_expand(N, synth.brownian_tt_cores(N, mus))
    assert U.shape[1] == math.factorial(D)
    t = agg.plan_tables(D, N, {D: U})
    u, Tp, Tq = int(t[4]), int(t[5]), int(t[6])
    assert (u, Tp, Tq) == (len(set(mus)), 1, len(set(mus)))
    colmap = 8 + D * U.shape[1]
    assert int(t[colmap]) == D and int(t[colmap + 1]) == math.factorial(D)   # one term, multiplicity D!


def test_tt_expand_errors():
    cores = synth.brownian_tt_cores(8, [0.5, -0.5])
    bad = [c.copy() for c in cores]
    bad[0] = np.concatenate([bad[0], bad[0]], axis=0)          # r_0 = 2
    with pytest.raises(agg.AggError) as e:
        agg.tt_expand(8, bad)
    assert e.value.status == agg.AGG_EINVAL
    nan = [c.copy() for c in cores]
    nan[1][0, 3, 0] = np.nan
    with pytest.raises(agg.AggError) as e:
        agg.tt_expand(8, nan)
    assert e.value.status == agg.AGG_ENONFINITE


def test_tt_expand_refuses_a_path_explosion():
    """Dense cores of ranks 128 x 128 x 128 over five modes have 2^21 paths."""
    N = 2
    ranks = [1, 128, 128, 128, 1]
    cores = [np.ones((ranks[m], N, ranks[m + 1])) for m in range(4)]
    with pytest.raises(agg.AggError) as e:
        agg.tt_expand(N, cores)
    assert e.value.status == agg.AGG_EUNSUPPORTED


# ---- oracle pins for kernels in tensor-train form --------------------------

def _random_cores(rng, N, ranks, positive=False):
    lo = 0.1 if positive else -1.0
    return [rng.uniform(lo, 1.0, size=(ranks[m], N, ranks[m + 1])) for m in range(len(ranks) - 1)]


def test_oracle_tt_full_of_diagonal_cores_is_the_cp_tensor():
    """A CP kernel of rank R is a TT kernel with ranks R whose inner cores are
    diagonal: the oracle's contraction must give the CP tensor built here
    directly from its definition."""
    import oracle
    rng = np.random.default_rng(21)
    N, R, d = 5, 3, 3
    U = rng.uniform(-1, 1, size=(d, R, N))
    cores = [np.zeros((1, N, R)), np.zeros((R, N, R)), np.zeros((R, N, 1))]
    for r in range(R):
        cores[0][0, :, r] = U[0, r]
        cores[1][r, :, r] = U[1, r]
        cores[2][r, :, 0] = U[2, r]
    assert np.abs(oracle.tt_full(cores) - dense_from_cp(U, N)).max() <= 1e-15


def test_oracle_tt_paths_reproduce_the_contraction():
    import oracle
    rng = np.random.default_rng(22)
    N = 5
    cores = _random_cores(rng, N, [1, 2, 3, 1])
    U = oracle.tt_paths(cores)
    assert U.shape == (3, 6, N)
    assert np.abs(dense_from_cp(U, N) - oracle.tt_full(cores)).max() <= 1e-14


def test_oracle_rhs_dense_equals_the_literal_cp_sums():
    """rhs_dense on the dense tensors of a CP kernel set equals rhs_direct (the
    literal sums over the CP form, in C)."""
    import oracle
    rng = np.random.default_rng(23)
    D, N = 4, 7
    kernel = {2: rng.uniform(0, 1, size=(2, 2, N)), 3: rng.uniform(0, 1, size=(3, 3, N)),
              4: rng.uniform(0, 1, size=(4, 2, N))}
    n = rng.uniform(0, 1, size=N)
    p, q = oracle.rhs_dense(D, N, {d: dense_from_cp(U, N) for d, U in kernel.items()}, n)
    pr, qr = oracle.rhs_direct(D, N, kernel, n)
    pr, qr = pr.sum(axis=0), qr.sum(axis=0)
    assert np.abs(p - pr).max() <= 1e-14 * np.abs(pr).max()
    assert np.abs(q - qr).max() <= 1e-14 * np.abs(qr).max()


# ---- integer tables of tensor-train plans ----------------------------------

def test_tt_tables_hand_derived():
    """D=2, N=3, one order-2 term with ranks (1, 2, 1); core 2's second column
    equals core 1's first.  L = 16 (max(16, 2^ceil(log2 5))), M = 8 -> M1 = 4,
    M2 = 2, g = 2; ids: core 1 [0, 1], core 2 [2, 0]; u = 3; one chunk of
    columns [0, 1, 2] holding cores [0, 1]."""
    c1 = np.array([1.0, 2.0, 3.0])
    c2 = np.array([0.5, 0.25, 0.125])
    c3 = np.array([4.0, 5.0, 6.0])
    core1 = np.zeros((1, 3, 2)); core1[0, :, 0] = c1; core1[0, :, 1] = c2
    core2 = np.zeros((2, 3, 1)); core2[0, :, 0] = c3; core2[1, :, 0] = c1
    want = [16, 4, 2, 2, 3, 1, 2, 2, 2,
            0, 1, 1, 2, 0, 1,
            0, 2, 2, 1, 2, 0,
            1, 3, 2, 0, 1, 2, 0, 1]
    got = agg.plan_tables_tt(2, 3, {2: [core1, core2]})
    assert got.tolist() == want


def test_tt_tables_mixed_radix_hand_derived():
    """D=3, N=65536, one order-3 term with ranks (1,1,1,1) and 3 distinct
    columns.  Power of two: L = 2^18, M = 2^17 -> M1 = 512, M2 = 256, g = 2.
    Mixed radix: X2 gives L' = 3 2^16 = 196608 (5 2^16 = 327680 is longer),
    M = 98304; X6: M2 = 256 (256^2 <= 98304 < 512^2), M1 = 384, no widening
    (3*2*256*16 = 24576 <= 64 KiB), 2^9 divides L'; X7: g = 2 (1024 // 384 = 2).
    Chunk capacity at M2 = 256: 151552 // (2*272*16) = 17, one chunk."""
    N = 65536
    cols = [np.full(N, v) for v in (1.0, 2.0, 3.0)]
    cores = [c.reshape(1, N, 1) for c in cols]
    tail = [1, 3, 3, 3, 0, 1, 1, 1, 0, 0, 2, 1, 1, 1, 0, 3, 1, 1, 2, 1, 3, 3, 0, 1, 2, 0, 1, 2]
    assert agg.plan_tables_tt(3, N, {3: cores}).tolist() == [262144, 512, 256, 2, 3] + tail
    assert agg.plan_tables_tt(3, N, {3: cores}, mixed=True).tolist() == [196608, 384, 256, 2, 3] + tail


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("case", range(6))
def test_tt_tables_match_the_twin(case, mixed):
    import oracle
    rng = np.random.default_rng(100 + case)
    D = [2, 3, 4, 4, 3, 4][case]
    N = [9, 40, 33, 257, 4096, 65536][case]
    prec = ["fp64", "fp32", "fp32c", "fp64", "fp32c", "fp64"][case]
    tt = {}
    for d in range(2, D + 1):
        ranks = [1] + [int(rng.integers(1, 7 if case < 5 else 7)) for _ in range(d - 1)] + [1]
        cores = _random_cores(rng, N, ranks)
        if d == 3 and ranks[1] > 1:
            cores[1][1, :, 0] = 0.0                       # an all-zero column
        if d == D and ranks[1] > 1:
            cores[0][0, :, 1] = cores[0][0, :, 0]          # a duplicate within a core
        if d > 2 and 2 in tt:
            cores[-1][0, :, 0] = tt[2][1][0, :, 0]        # shared with another order
        tt[d] = cores
    got = agg.plan_tables_tt(D, N, tt, prec, mixed=mixed)
    want = oracle.plan_tables_tt(D, N, tt, prec, mixed=mixed)["flat"]
    assert got.tolist() == want.tolist()
