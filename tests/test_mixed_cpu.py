"""Mixed-radix transform lengths (3 2^a and 5 2^a) on the CPU.

* The reading behind them: any cyclic length L >= De N - 1 keeps the gain
  outputs k in [2, N] free of wrap-around, whatever L's factors (Sec. 2's
  convolution via the FFT only needs L past the last index the d-fold product
  reaches).  Checked with numpy's FFT at lengths 3 2^a and 5 2^a against the
  oracle's literal sums.
* The oracle's written rules X2/X6/X7 at hand-derived sizes.
* The library's planner against those rules, bit for bit.
* The library's binary64 roots of unity at the mixed lengths, within 1 ulp.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle.plan import plan_tables as oracle_plan
from oracle.twiddle import twiddles_ref


def _gain_cyclic(D, N, kernel, n, L):
    """p^(d) via length-L cyclic convolutions of the weighted columns (numpy FFT)."""
    p = np.zeros((D + 1, N))
    for d, U in kernel.items():
        acc = np.zeros(L)
        for r in range(U.shape[1]):
            spec = np.ones(L, dtype=complex)
            for m in range(d):
                x = np.zeros(L)
                x[:N] = U[m, r] * n
                spec *= np.fft.fft(x)
            acc += np.fft.ifft(spec).real
        # index s - d of the d-fold product is total size s
        fact = float(np.prod(np.arange(1, d + 1)))
        for k in range(1, N + 1):
            if k - d >= 0:
                p[d, k - 1] = acc[k - d] / fact
    return p


@pytest.mark.parametrize("D,N,L", [(3, 16, 48), (3, 32, 96), (2, 40, 80), (4, 20, 80), (5, 48, 240)])
def test_cyclic_length_with_odd_factor_has_no_wraparound(D, N, L):
    assert L >= D * N - 1
    k = synth.kernel_random(D, N, 2, 3)
    n = synth.n0_random_dense(N, 4)
    p_ref, _ = oracle.rhs_direct(D, N, k, n)
    p = _gain_cyclic(D, N, k, n, L)
    scale = np.max(np.abs(p_ref))
    assert np.max(np.abs(p[2:] - p_ref[2:])) <= 1e-13 * scale
    # one index shorter wraps: the largest size's gain then picks up aliased mass
    if L - 1 < D * N - 1:
        pw = _gain_cyclic(D, N, k, n, L - 1)
        assert np.max(np.abs(pw[D] - p_ref[D])) > 1e-6 * scale


def _k(D, N, kind, seed=0, R=1):
    return {"additive": lambda: synth.kernel_additive(D, N),
            "brownian": lambda: synth.kernel_brownian_sum(D, N),
            "random": lambda: synth.kernel_random(D, N, R, seed),
            "constant": lambda: synth.kernel_constant(D, N)}[kind]()


# (D, N, kernel, ranks, expected (L, M1, M2, g)) derived by hand from X2/X6/X7
HAND = [
    # 3 4096 - 1 = 12287 <= 48 2^8 = 12288 < 2^14; M = 6144, M2 = 64 (64^2 <= 6144 < 128^2), M1 = 96,
    # g = largest power of two <= min(64, 1024 // 96 = 10) = 8
    (3, 4096, "brownian", 1, (12288, 96, 64, 8)),
    # 2 10240 - 1 = 20479 <= 80 2^8 = 20480 < 48 2^9 and < 2^15; M = 10240, M2 = 64, M1 = 160, g = 4
    (2, 10240, "random", 1, (20480, 160, 64, 4)),
    # D = 5, N = 2^20: L = 80 2^16 = 5 2^20 (48 2^17 = 3 2^20 is longer); M = 5 2^19,
    # M2 = 1024, M1 = 2560 > 1280 -> M1 = 1280, M2 = 2048; g = 1
    (5, 1 << 20, "additive", 1, (5 << 20, 1280, 2048, 1)),
    # D = 3, N = 2^19: L = 48 2^15 = 3 2^19; M = 3 2^18, M2 = 512, M1 = 1536; g = 1
    (3, 1 << 19, "brownian", 1, (3 << 19, 1536, 512, 1)),
    # 35 distinct columns (rank 7 at d = 2, 3) at 3 4096: 35 2 64 16 > 64 KiB -> M1 = 192,
    # M2 = 32, g = largest power of two <= min(32, 5) = 4
    (3, 4096, "random", 7, (12288, 192, 32, 4)),
    # C1 size: 3 64 - 1 = 191 <= 192 < 256 but M = 96 gives M1 = 12 < 96: the power of two
    (3, 64, "constant", 1, (256, 16, 8, 8)),
    # 2 2048 - 1 = 4095: the power of two 4096 is shorter than 48 2^7 = 6144;
    # M = 2048, M1 = 2^6, M2 = 32, g = min(32, 16)
    (2, 2048, "random", 1, (4096, 64, 32, 16)),
]


@pytest.mark.parametrize("D,N,kind,R,want", HAND)
def test_oracle_mixed_rules_by_hand(D, N, kind, R, want):
    t = oracle_plan(D, N, _k(D, N, kind, 5, R), "fp64", mixed=True)
    assert (t["L"], t["M1"], t["M2"], t["g"]) == want
    assert 2 * t["M1"] * t["M2"] == t["L"]
    # without the option: the power-of-two rules
    t2 = oracle_plan(D, N, _k(D, N, kind, 5, R), "fp64")
    assert t2["L"] & (t2["L"] - 1) == 0
    if want[0] & (want[0] - 1) == 0:
        assert np.array_equal(t["flat"], t2["flat"])


agg = pytest.importorskip("paper_1905_09071_amd")


@pytest.mark.parametrize("D,N,kind,R,want", HAND)
@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32c"])
def test_planner_mixed_bit_exact_by_hand(D, N, kind, R, want, prec):
    k = _k(D, N, kind, 5, R)
    ref = oracle_plan(D, N, k, prec, mixed=True)["flat"]
    got = agg.plan_tables(D, N, k, prec, mixed=True)
    assert np.array_equal(got, ref)


def _sweep():
    rng = np.random.default_rng(11)
    cases = []
    for _ in range(60):
        D = int(rng.integers(2, 6))
        N = int(rng.integers(1, 200000))
        R = int(rng.integers(1, 9))
        cases.append((D, N, R, int(rng.integers(0, 1000))))
    return cases


@pytest.mark.parametrize("D,N,R,seed", _sweep())
def test_planner_mixed_bit_exact_sweep(D, N, R, seed):
    """Random sizes: every outcome (3 2^a, 5 2^a, fallback to 2^a, chunked rows,
    unsupported) agrees with the oracle's rules."""
    k = synth.kernel_random(D, N, R, seed)
    for prec in ("fp64", "fp32"):
        try:
            ref = oracle_plan(D, N, k, prec, mixed=True)["flat"]
        except ValueError:
            with pytest.raises(agg.AggError):
                agg.plan_tables(D, N, k, prec, mixed=True)
            continue
        got = agg.plan_tables(D, N, k, prec, mixed=True)
        assert np.array_equal(got, ref)


def test_mixed_and_plain_options_refused_together():
    k = synth.kernel_constant(3, 64)
    with pytest.raises(agg.AggError) as e:
        agg.plan_tables(3, 64, k, "fp64", plain=True, mixed=True)
    assert e.value.status == agg.AGG_EINVAL


@pytest.mark.parametrize("P", [24, 40, 96, 160, 1536, 1280])
def test_mixed_twiddles_within_one_ulp(P):
    got = agg.twiddles(P)
    ref = twiddles_ref(P)
    ulp = np.spacing(np.maximum(np.abs(ref), 1e-300))
    assert np.all(np.abs(got - ref) <= ulp)
    # exact symmetries: w^(P/4) = -i, w^(P/8) on the diagonal, w^(P/2) = -1
    assert got[P // 4, 0] == 0.0 and got[P // 4, 1] == -1.0
    assert got[P // 8, 0] == -got[P // 8, 1]
    assert got[P // 2, 0] == -1.0 and got[P // 2, 1] == 0.0


@pytest.mark.parametrize("P", [3 << 19, 5 << 20])
def test_mixed_twiddles_sampled_large(P):
    got = agg.twiddles(P)
    idx = list(np.random.default_rng(1).integers(0, P, 200)) + [P // 3, 2 * P // 3] if P % 3 == 0 else \
        list(np.random.default_rng(1).integers(0, P, 200)) + [P // 5, 2 * P // 5]
    ref = twiddles_ref(P, idx)
    ulp = np.spacing(np.maximum(np.abs(ref), 1e-300))
    assert np.all(np.abs(got[idx] - ref) <= ulp)


@pytest.mark.parametrize("P", [3, 6, 12, 7, 0, 80 * 3])
def test_twiddles_refuse_other_lengths(P):
    with pytest.raises(agg.AggError):
        agg.twiddles(P)
