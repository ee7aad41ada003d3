"""Pins for the oracle's written plan rules (CPU only): tables derived by hand
for the benchmark kernels, and the edge cases of the rules."""
import numpy as np
import pytest

import synth
from oracle.plan import plan_tables, Unsupported


def test_ballistic_d4_tables():
    """C^(d) = sum_{m!=l} (i_m/i_l)^a, D = 4.  Scanning d=2 mode 1 meets i^a (id 0)
    then i^-a (id 1); d=3 mode 1 first meets the all-ones column (id 2).
    Gain: d=2 -> {0,1} x2; d=3 -> {0,1,2} x6; d=4 -> {0,1,2,2} x12."""
    t = plan_tables(4, 65536, synth.kernel_ballistic(4, 65536, 0.4), "fp64")
    assert (t["L"], t["M1"], t["M2"], t["g"], t["u"], t["De"]) == (1 << 18, 512, 256, 2, 3, 4)
    assert t["pterms"] == [((0, 1), 2), ((0, 1, 2), 6), ((0, 1, 2, 2), 12)]
    assert t["qterms"] == [((2, 0, (1,)), 1), ((2, 1, (0,)), 1),
                           ((3, 0, (1, 2)), 2), ((3, 1, (0, 2)), 2), ((3, 2, (0, 1)), 2),
                           ((4, 0, (1, 2, 2)), 3), ((4, 1, (0, 2, 2)), 3), ((4, 2, (0, 1, 2)), 6)]


def test_brownian_sum_d3_tables():
    """(sum_m i_m^mu)(sum_l i_l^-mu): the m == l terms are exact ones."""
    t = plan_tables(3, 4096, synth.kernel_brownian_sum(3, 4096), "fp64")
    assert (t["L"], t["u"]) == (16384, 3)
    assert t["pterms"] == [((0, 0), 2), ((1, 2), 2), ((0, 0, 0), 3), ((0, 1, 2), 6)]


def test_constant_kernel_tables():
    t = plan_tables(3, 64, synth.kernel_constant(3, 64), "fp64")
    assert (t["L"], t["M1"], t["M2"], t["g"], t["u"]) == (256, 16, 8, 8, 1)
    assert t["pterms"] == [((0, 0), 1), ((0, 0, 0), 1)]
    assert t["qterms"] == [((2, 0, (0,)), 1), ((3, 0, (0, 0)), 1)]


def test_dedup_is_bitwise():
    k = synth.kernel_constant(2, 10)
    k[2][1, 0, 3] = np.nextafter(1.0, 2.0)
    t = plan_tables(2, 10, k)
    assert t["u"] == 2 and t["colmap"] == [0, 1]


def test_length_rule_edges():
    # L >= D*N - 1 keeps outputs 2..N clear of wrap-around; D=3, N=2 needs L=8 (not 4)
    assert plan_tables(3, 2, synth.kernel_constant(3, 2))["L"] == 16
    assert plan_tables(3, 6, synth.kernel_constant(3, 6))["L"] == 32
    assert plan_tables(4, 65536, synth.kernel_constant(4, 65536))["L"] == 1 << 18
    # effective order: a rank-0 top order does not lengthen the transform
    k = synth.kernel_constant(4, 1000)
    k[4] = np.zeros((4, 0, 1000))
    assert plan_tables(4, 1000, k)["De"] == 3
    assert plan_tables(4, 1000, k)["L"] == 4096


def test_split_rule_and_unsupported():
    t = plan_tables(5, 1 << 20, synth.kernel_additive(5, 1 << 20), "fp64")
    assert (t["L"], t["M1"], t["M2"], t["u"]) == (1 << 23, 2048, 2048, 2)
    with pytest.raises(Unsupported):
        plan_tables(5, 1 << 20, synth.kernel_random(5, 1 << 20, 1, 0), "fp64")
