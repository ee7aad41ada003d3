"""TT-cross compression of kernels given as functions (host, no GPU): the
train must reproduce kernels of known low TT rank exactly (separable, and the
generalized Brownian kernels of Sec. 2 with ranks C(D, lambda)), approximate
a non-separable kernel (the ballistic kernel of binary aggregation and a
three-particle generalization) to the error it reports, checked against the
function on the whole index grid, and refuse bad arguments."""
import itertools
import math

import numpy as np
import pytest

import oracle

agg = pytest.importorskip("paper_1905_09071_amd")


def grid(d, N):
    return np.array(list(itertools.product(range(1, N + 1), repeat=d)), dtype=np.int64)


def brownian(mus):
    def f(a):
        s = a.astype(np.float64)
        out = np.zeros(len(a))
        for sg in itertools.permutations(range(len(mus))):
            out += np.prod([s[:, sg[j]] ** mus[j] for j in range(len(mus))], axis=0)
        return out
    return f


def ballistic(a):
    """sum-of-cube-roots squared times the square root of the summed inverse
    sizes: for d = 2 the ballistic collision kernel of binary aggregation."""
    s = a.astype(np.float64)
    return np.sum(s ** (1 / 3), axis=1) ** 2 * np.sqrt(np.sum(1.0 / s, axis=1))


def test_separable_kernel_is_rank_one():
    N = 40
    f = lambda a: (a[:, 0] ** 0.5) * (a[:, 1] ** -0.3) * (a[:, 2] ** 0.2)
    cores, err = agg.tt_cross(3, N, f, tol=1e-13, rmax=4, seed=1)
    assert [c.shape[2] for c in cores[:-1]] == [1, 1]
    full = oracle.tt_full(cores)
    ref = f(grid(3, N)).reshape((N,) * 3)
    assert np.abs(full - ref).max() <= 1e-13 * np.abs(ref).max()
    assert err <= 1e-13


@pytest.mark.parametrize("mus", [[0.3, -0.3, 0.1], [0.5, -0.2, 0.1, -0.4]])
def test_brownian_kernels_are_recovered_with_their_ranks(mus):
    D = len(mus)
    N = 16 if D == 3 else 9
    cores, err = agg.tt_cross(D, N, brownian(mus), tol=1e-12, rmax=8, seed=2)
    ranks = [1] + [c.shape[2] for c in cores]
    assert all(ranks[m] <= math.comb(D, m) for m in range(D + 1))
    full = oracle.tt_full(cores)
    ref = brownian(mus)(grid(D, N)).reshape((N,) * D)
    e = np.abs(full - ref).max() / np.abs(ref).max()
    assert e <= 1e-12 and err <= 1e-12


def test_ballistic_kernel_to_its_reported_error():
    N = 1024
    cores, err = agg.tt_cross(2, N, ballistic, tol=1e-12, rmax=8, seed=3)
    A = cores[0][0] @ cores[1][:, :, 0]
    i = np.arange(1, N + 1, dtype=np.float64)
    ref = (i[:, None] ** (1 / 3) + i[None, :] ** (1 / 3)) ** 2 * np.sqrt(1 / i[:, None] + 1 / i[None, :])
    e = np.abs(A - ref).max() / ref.max()
    assert cores[0].shape[2] == 8
    assert e <= 1e-5
    assert err <= 1e-5 and e <= 20 * err      # the sample estimate is representative of the grid
    # a lower rank is less accurate
    c4, err4 = agg.tt_cross(2, N, ballistic, tol=1e-12, rmax=4, seed=3)
    assert err4 > err


def test_three_particle_ballistic_kernel():
    D, N = 3, 24
    cores, err = agg.tt_cross(D, N, ballistic, tol=1e-12, rmax=8, seed=4)
    full = oracle.tt_full(cores)
    ref = ballistic(grid(D, N)).reshape((N,) * D)
    e = np.abs(full - ref).max() / ref.max()
    assert e <= 1e-4 and e <= 20 * max(err, 1e-16)


def test_tt_cross_refusals():
    f = lambda a: np.ones(len(a))
    with pytest.raises(agg.AggError) as e:
        agg.tt_cross(2, 10, f, rmax=9)
    assert e.value.status == agg.AGG_EINVAL
    with pytest.raises(agg.AggError) as e:
        agg.tt_cross(2, 10, lambda a: np.full(len(a), np.nan))
    assert e.value.status == agg.AGG_ENONFINITE
