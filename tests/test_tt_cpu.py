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
