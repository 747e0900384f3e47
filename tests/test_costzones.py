"""The numpy cost-zone split the GPU tests compare bh_shard_bounds with, against the literal
definition and against splits worked by hand.  CPU only."""
import numpy as np

from tests.costzones import cost_zones, cost_zones_literal, group_zones


def test_by_hand():
    # costs 1..4 (T = 10), two ranges: the first rank with 2 P(r) >= 10 is r = 3 (P = 6)
    assert cost_zones([1, 2, 3, 4], 2).tolist() == [0, 3, 4]
    # equal costs: range j starts at ceil(j n / G)
    assert cost_zones([1] * 10, 3).tolist() == [0, 4, 7, 10]
    # more ranges than bodies: empty ranges where a boundary repeats
    assert cost_zones([5, 1], 4).tolist() == [0, 1, 1, 1, 2]


def test_search_is_the_definition():
    rng = np.random.default_rng(5)
    for n in (1, 2, 7, 100, 1000):
        c = rng.integers(1, 50, n)
        for G in (1, 2, 3, 8, 13, 64):
            assert np.array_equal(cost_zones(c, G), cost_zones_literal(c, G)), (n, G)


def test_group_split_by_hand():
    # 130 bodies in groups of 64, 64 and 2; group costs 10, 0, 0 -> 74, 64, 2 (T = 140)
    # two ranges: 2 P(x) >= 140 first at x = 1 (P = 74): the split is at rank 64
    assert group_zones([10, 0, 0], 130, 2).tolist() == [0, 64, 130]
    # heavy last group: P = 64, 128, 1130; half of T (565) is reached at x = 3 -> rank min(192, 130)
    assert group_zones([0, 0, 1000], 130, 2).tolist() == [0, 130, 130]
