"""The C-ABI library without a GPU: it loads, exports every symbol of
include/agg.h, its host planner reproduces the oracle's written plan rules bit
for bit, its binary64 twiddles are within 1 ulp of the correctly rounded
values, and invalid arguments are refused before any device call."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import synth
from oracle.plan import plan_tables as oracle_plan
from oracle.twiddle import twiddles_ref
from conftest import unweighted_modes

agg = pytest.importorskip("paper_1905_09071_amd")
from paper_1905_09071_amd import _lib  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "agg.h")).read()
    declared = set(re.findall(r"\b(agg_\w+)\s*\(", hdr))
    assert declared, "no declarations found"
    L = _lib.lib()
    for name in declared:
        assert hasattr(L, name), f"libagg.so does not export {name}"
    assert declared == {e[0] for e in _lib.EXPORTS}


KERNELS = [
    ("constant", lambda D, N: synth.kernel_constant(D, N)),
    ("ballistic", lambda D, N: synth.kernel_ballistic(D, N, 0.4)),
    ("ballistic0", lambda D, N: synth.kernel_ballistic(D, N, 0.0)),
    ("brownian", lambda D, N: synth.kernel_brownian_sum(D, N)),
    ("additive", lambda D, N: synth.kernel_additive(D, N)),
    ("random", lambda D, N: synth.kernel_random(D, N, 2, 7)),
    ("gbrown", lambda D, N: {D: synth.kernel_generalized_brownian(N, [0.3, -0.3, 0.1, 0.0][:D])}),
]


@pytest.mark.parametrize("kname,kf", KERNELS)
@pytest.mark.parametrize("D,N", [(2, 1), (2, 5), (3, 2), (3, 64), (4, 37), (4, 1000), (3, 4096), (4, 65536)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32c"])
def test_plan_tables_bit_exact(kname, kf, D, N, prec):
    if kname == "gbrown" and D > 4:
        pytest.skip("mu list has 4 entries")
    k = kf(D, N)
    try:
        ref = oracle_plan(D, N, k, prec)["flat"]
    except ValueError:
        with pytest.raises(agg.AggError):
            agg.plan_tables(D, N, k, prec)
        return
    got = agg.plan_tables(D, N, k, prec)
    assert got.dtype == np.int64 and np.array_equal(got, ref)


@pytest.mark.parametrize("kname,kf", KERNELS[:5])
def test_plain_plan_tables_bit_exact(kname, kf):
    """Without column sharing every (d, m, r) column gets its own id."""
    k = kf(4, 100)
    ref = oracle_plan(4, 100, k, "fp64", dedup=False)
    got = agg.plan_tables(4, 100, k, "fp64", plain=True)
    assert np.array_equal(got, ref["flat"])
    assert ref["u"] == sum(d * k[d].shape[1] for d in k)


def test_plan_tables_large_and_unsupported():
    k = synth.kernel_additive(5, 1 << 20)
    assert np.array_equal(agg.plan_tables(5, 1 << 20, k), oracle_plan(5, 1 << 20, k)["flat"])
    kr = synth.kernel_random(5, 1 << 20, 1, 0)
    with pytest.raises(agg.AggError) as e:
        agg.plan_tables(5, 1 << 20, kr)
    assert e.value.status == agg.AGG_EUNSUPPORTED


@pytest.mark.parametrize("P", [2, 4, 8, 16, 256, 2048])
def test_twiddles_within_one_ulp(P):
    got = agg.twiddles(P)
    ref = twiddles_ref(P)
    ulp = np.spacing(np.maximum(np.abs(ref), 1e-300))
    assert np.all(np.abs(got - ref) <= ulp)
    # exact symmetries of the roots of unity
    assert got[0, 0] == 1.0 and got[0, 1] == 0.0
    if P >= 4:
        assert got[P // 4, 0] == 0.0 and got[P // 4, 1] == -1.0
    if P >= 8:
        assert got[P // 8, 0] == -got[P // 8, 1]


def test_twiddles_sampled_large():
    P = 1 << 23
    got = agg.twiddles(P)
    idx = list(np.random.default_rng(0).integers(0, P, 300))
    ref = twiddles_ref(P, idx)
    ulp = np.spacing(np.maximum(np.abs(ref), 1e-300))
    assert np.all(np.abs(got[idx] - ref) <= ulp)


def _create(D, N, kernel, prec=0, batch=1):
    terms, nt, keep = agg.make_terms(D, N, kernel) if kernel is not None else (None, 0, [])
    h = ctypes.c_void_p()
    rc = _lib.lib().agg_plan_create(D, N, terms, nt, prec, batch, None, ctypes.byref(h))
    return rc


def test_invalid_arguments_refused_before_any_device_call():
    L = _lib.lib()
    k = synth.kernel_constant(3, 8)
    assert _create(1, 8, k) == agg.AGG_EINVAL          # D < 2
    assert _create(9, 8, {}) == agg.AGG_EINVAL         # D > AGG_MAX_D
    assert _create(3, 0, {}) == agg.AGG_EINVAL         # N < 1
    assert _create(3, 8, k, prec=7) == agg.AGG_EINVAL  # unknown precision
    assert _create(3, 8, k, batch=0) == agg.AGG_EINVAL
    assert _create(2, 8, k) == agg.AGG_EINVAL          # a term of order 3 > D
    kb = synth.kernel_constant(3, 8)
    kb[3] = kb[3].copy()
    kb[3][1, 0, 2] = np.nan
    assert _create(3, 8, kb) == agg.AGG_ENONFINITE
    assert b"non-finite" in L.agg_last_error()
    # duplicate order and negative rank, built by hand
    terms = (_lib.agg_term * 2)()
    col = np.ones(8)
    for t in range(2):
        terms[t].d = 2
        terms[t].rank = 1
        for m in range(2):
            terms[t].U[m] = col.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p()
    assert L.agg_plan_create(3, 8, terms, 2, 0, 1, None, ctypes.byref(h)) == agg.AGG_EINVAL
    assert b"duplicate" in L.agg_last_error()
    terms[0].rank = -1
    assert L.agg_plan_create(3, 8, terms, 1, 0, 1, None, ctypes.byref(h)) == agg.AGG_EINVAL
    terms[0].rank = 1
    terms[0].U[1] = ctypes.POINTER(ctypes.c_double)()
    assert L.agg_plan_create(3, 8, terms, 1, 0, 1, None, ctypes.byref(h)) == agg.AGG_EINVAL
    assert L.agg_plan_create(3, 8, terms, 1, 0, 1, None, None) == agg.AGG_EINVAL
    # length limit: 4*N - 1 > 2^23 is refused before any column is read
    Nbig = (1 << 21) + 1
    big = {4: np.ones((4, 1, Nbig))}
    assert _create(4, Nbig, big) == agg.AGG_EUNSUPPORTED
    assert b"2^23" in L.agg_last_error()
    assert _create(3, 8, k, prec=0x400) == agg.AGG_EINVAL   # unknown option bit
    assert _create(3, 8, k, prec=0x300) == agg.AGG_EINVAL   # AGG_PLAIN with AGG_MIXED_RADIX


def test_null_plan_calls_are_refused():
    L = _lib.lib()
    assert L.agg_rhs(None, None, None) == agg.AGG_EINVAL
    assert L.agg_rk2_step(None, None, 1e-3) == agg.AGG_EINVAL
    assert L.agg_solve(None, None, 1e-3, 1.0, None) == agg.AGG_EINVAL
    assert L.agg_plan_destroy(None) == agg.AGG_OK
    assert L.agg_poll(None, 1, None, None) == agg.AGG_EINVAL
    assert L.agg_engine_destroy(None) == agg.AGG_OK


# ---- row-pass chunks and host kernel compression --------------------------------

def _expsum_kernel(D, N, R=31, weighted=False):
    f = synth.sum_kernel_values(2, D * N)
    alpha, w, err = agg.expsum_fit(f, 2, R)
    return synth.kernel_expsum(D, N, alpha, w, weighted), err / f.max()


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("D,N,prec", [(5, 65536, "fp64"), (5, 65536, "fp32"), (5, 1 << 20, "fp32c"),
                                      (5, 1 << 20, "fp32")])
def test_chunked_plan_tables_bit_exact(D, N, prec, weighted):
    """The chunk rule on the compressed (sum_m i_m)^(1/2) kernel: 64 distinct
    columns (two per rank-one term) with the weights in mode-1 columns, 32
    with the weights given as term weights."""
    k, _ = _expsum_kernel(D, N, weighted=weighted)
    kk = unweighted_modes(k)
    ref = oracle_plan(D, N, kk, prec)
    assert ref["u"] == (32 if weighted else 64)
    got = agg.plan_tables(D, N, k, prec)
    assert np.array_equal(got, ref["flat"])
    M2, cs = ref["M2"], 8 if prec == "fp32" else 16
    if ref["u"] * 2 * (M2 + M2 // 16) * cs + (M2 * cs if M2 <= 512 else 0) > 147456:
        assert len(ref["chunks"]) >= 2
        for cols, terms in ref["chunks"]:
            assert len(cols) <= 151552 // (2 * (M2 + M2 // 16) * cs)
    else:
        assert ref["chunks"] == []


def test_chunked_plan_tables_random_kernel():
    """Chunks of a kernel without shared columns (terms of 2, 3 and 4 columns)."""
    D, N = 4, 65536
    k = synth.kernel_random(D, N, {2: 4, 3: 8, 4: 11}, 21)
    ref = oracle_plan(D, N, k, "fp64")
    assert ref["u"] == 76 and len(ref["chunks"]) == 2
    assert np.array_equal(agg.plan_tables(D, N, k, "fp64"), ref["flat"])
    covered = sorted(t for _, terms in ref["chunks"] for t in terms)
    assert covered == list(range(len(ref["pterms"])))


def test_expsum_fit_rank32_sqrt_sum_kernel():
    """(i_1+..+i_5)^(1/2) for N = 2^20: rank 32 (31 exponentials and a constant)
    within 1e-8 of max C over every reachable total size, the reported error
    being the true maximum (re-evaluated here independently)."""
    D, N = 5, 1 << 20
    f = synth.sum_kernel_values(2, D * N)
    alpha, w, err = agg.expsum_fit(f, 2, 31)
    assert alpha.size == 31 and w.size == 32 and np.all(alpha > 0) and np.all(np.diff(alpha) > 0)
    assert err <= 1e-8 * f.max()
    s = np.arange(2, D * N + 1, dtype=np.float64)
    worst = 0.0
    for i0 in range(0, s.size, 1 << 18):
        ss = s[i0:i0 + (1 << 18)]
        v = w[0] + np.exp(-np.outer(ss, alpha)) @ w[1:]
        worst = max(worst, float(np.max(np.abs(v - f[i0:i0 + (1 << 18)]))))
    assert abs(worst - err) <= 1e-6 * err
    # the factors reproduce the function of the total size at sampled multi-indices
    k = synth.kernel_expsum(D, 4096, alpha, w)
    rng = np.random.default_rng(5)
    for d in (2, 5):
        U = k[d]
        for _ in range(20):
            idx = rng.integers(1, 4097, size=d)
            c = sum(np.prod([U[m][r, idx[m] - 1] for m in range(d)]) for r in range(32))
            assert abs(c - math.sqrt(idx.sum())) <= err + 1e-12 * np.abs(w).sum()


def test_expsum_fit_special_cases_and_errors():
    f = np.full(1000, 2.5)
    alpha, w, err = agg.expsum_fit(f, 1, 0)
    assert alpha.size == 0 and w[0] == pytest.approx(2.5, abs=1e-12) and err <= 1e-12
    # 1/s (completely monotone) converges geometrically in the number of terms
    s = np.arange(1, 10001, dtype=np.float64)
    errs = [agg.expsum_fit(1.0 / s, 1, R)[2] for R in (8, 16, 24)]
    assert errs[1] <= 0.1 * errs[0] and errs[2] <= 0.1 * errs[1] and errs[2] <= 1e-7
    with pytest.raises(agg.AggError) as e:
        agg.expsum_fit(f, 0, 4)
    assert e.value.status == agg.AGG_EINVAL
    with pytest.raises(agg.AggError) as e:
        agg.expsum_fit(f, 1, 65)
    assert e.value.status == agg.AGG_EINVAL
    with pytest.raises(agg.AggError) as e:      # 5 sizes cannot fix 9 weights
        agg.expsum_fit(np.ones(5), 1, 8)
    assert e.value.status == agg.AGG_EINVAL
    g = f.copy()
    g[7] = np.nan
    with pytest.raises(agg.AggError) as e:
        agg.expsum_fit(g, 1, 4)
    assert e.value.status == agg.AGG_ENONFINITE


def test_expsum_fit_relative_error():
    """A relative fit bounds |fit - f| / |f| at every integer (checked here at
    all of them), and is refused for a vanishing f."""
    s = np.arange(2, 200001, dtype=np.float64)
    f = np.sqrt(s)
    alpha, w, err = agg.expsum_fit(f, 2, 24, relative=True)
    v = w[0] + np.exp(-np.outer(s, alpha)) @ w[1:]
    worst = float(np.max(np.abs(v - f) / f))
    assert abs(worst - err) <= 1e-6 * err and err <= 1e-7
    _, _, aerr = agg.expsum_fit(f, 2, 24)
    assert aerr / f.max() <= err      # the absolute fit is tighter relative to max f
    with pytest.raises(agg.AggError) as e:
        agg.expsum_fit(np.zeros(10), 1, 2, relative=True)
    assert e.value.status == agg.AGG_EINVAL


def test_term_weights_validation():
    k = synth.kernel_random(3, 50, 2, 1)
    kw = {d: {"U": U, "weight": np.array([0.5, -2.0])} for d, U in k.items()}
    assert np.array_equal(agg.plan_tables(3, 50, kw), agg.plan_tables(3, 50, k))
    bad = {d: {"U": U, "weight": np.array([0.5, np.inf])} for d, U in k.items()}
    with pytest.raises(agg.AggError) as e:
        agg.plan_tables(3, 50, bad)
    assert e.value.status == agg.AGG_ENONFINITE
    with pytest.raises(ValueError):
        agg.plan_tables(3, 50, {2: {"U": k[2], "weight": np.ones(3)}})


def test_chunked_plan_tables_shared_column():
    """A column shared by every term (the ones column) is listed in every
    chunk whose terms use it."""
    D, N = 4, 65536
    k = synth.kernel_random_first_mode(D, N, 25, 23)
    ref = oracle_plan(D, N, k, "fp64")
    assert ref["u"] == 76 and len(ref["chunks"]) >= 2
    assert np.array_equal(agg.plan_tables(D, N, k, "fp64"), ref["flat"])
    ones = 25
    assert sum(ones in cols for cols, _ in ref["chunks"]) >= 2


def test_chunk_rule_counts_padded_rows_and_twiddles():
    """u = 9 columns at M2 = 512 fill exactly 144 KiB unpadded; with the LDS
    padding and the row twiddles they do not, so the plan takes two chunks
    (the unchunked row pass would not fit a workgroup's LDS)."""
    D, N = 3, 1 << 19
    k = synth.kernel_random(D, N, {2: 3, 3: 1}, 31)
    ref = oracle_plan(D, N, k, "fp64")
    assert ref["u"] == 9 and ref["M2"] == 512 and len(ref["chunks"]) == 2
    assert np.array_equal(agg.plan_tables(D, N, k, "fp64"), ref["flat"])


def test_planner_refuses_rows_of_one_value():
    """More than 1024 distinct columns at L = 16: refused at planning (the row
    pass has no launch for rows of one value), as the oracle's twin refuses it."""
    k = synth.kernel_random(2, 2, 600, 3)
    with pytest.raises(agg.AggError) as e:
        agg.plan_tables(2, 2, k, "fp64")
    assert e.value.status == agg.AGG_EUNSUPPORTED
    k = synth.kernel_random(2, 2, 500, 3)
    assert np.array_equal(agg.plan_tables(2, 2, k, "fp64"), np.array(oracle_plan(2, 2, k, "fp64")["flat"]))
