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


def test_chunked_tables_by_hand():
    """D = 3, N = 2^19, random ranks R_2 = 3, R_3 = 1 (nine distinct columns).
    P2: L = 2^21 (3N - 1 = 1572863).  P6: 9*2*1024*16 B > 64 KiB at M1 = 1024,
    so M1 = 2048, M2 = 512 (the loop stops at M1 = 2048).  P7: g = 1.
    P8: rows 9*2*544*16 + 512*16 = 164864 B > 144 KiB, so chunks of
    cmax = floor(151552 / (2*544*16)) = 8 columns.  Gain terms {0,3}, {1,4},
    {2,5}, {6,7,8} in visiting order: the first three share a chunk of six
    columns; adding {6,7,8} would need nine, so it opens the second chunk."""
    N = 1 << 19
    t = plan_tables(3, N, synth.kernel_random(3, N, {2: 3, 3: 1}, 31), "fp64")
    assert (t["L"], t["M1"], t["M2"], t["g"], t["u"], t["De"]) == (1 << 21, 2048, 512, 1, 9, 3)
    assert t["colmap"] == list(range(9))
    assert t["pterms"] == [((0, 3), 1), ((1, 4), 1), ((2, 5), 1), ((6, 7, 8), 1)]
    assert t["qterms"] == [((2, 3, (0,)), 1), ((2, 4, (1,)), 1), ((2, 5, (2,)), 1), ((3, 8, (6, 7)), 1)]
    assert t["chunks"] == [([0, 1, 2, 3, 4, 5], [0, 1, 2]), ([6, 7, 8], [3])]


def test_too_many_columns_for_the_shortest_rows():
    """P6: 1200 distinct columns at L = 16 would leave rows of one value."""
    with pytest.raises(Unsupported):
        plan_tables(2, 2, synth.kernel_random(2, 2, 600, 3), "fp64")
    assert plan_tables(2, 2, synth.kernel_random(2, 2, 500, 3), "fp64")["M2"] == 2
