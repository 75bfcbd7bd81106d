"""Alg. 1 (pruning-level selection) and the usage-ranked keep mask, on
hand-built tables (host logic, no GPU).  Every hand table is checked on the
oracle's plain version (a pin of the oracle) and on the product's, and the
two are compared on random tables."""
import math

import numpy as np
import pytest

import oracle

prune = pytest.importorskip("paper_2512_20943_amd.prune")


@pytest.fixture(params=["oracle", "product"])
def select(request):
    return oracle.select_level if request.param == "oracle" else prune.select_level


@pytest.fixture(params=["oracle", "product"])
def keep_mask(request):
    return oracle.usage_keep_mask if request.param == "oracle" else prune.usage_keep_mask


def lowest_fitting(space, cands, C):
    """Reference by linear scan: the lowest candidate level with size <= C."""
    for i in cands:
        if space[i][1] <= C:
            return i
    return None


def test_no_cliff_selects_lowest_level_that_fits(select):
    space = [(40.0 - i, 1000 - 90 * i) for i in range(11)]  # steady 1 dB drops
    for C in (1000, 999, 730, 460, 100, 99):
        p = select(space, beta=2.0, bandwidth=C * 30.0, rate=30.0)
        exp = lowest_fitting(space, range(11), C)
        assert p == (exp if exp is not None else 10)


def test_quality_cliff_limits_the_candidates(select):
    # drops: -1, -1, -1, -5 (5 > 2 x 1: cliff at level 4)
    q = [40.0, 39.0, 38.0, 37.0, 32.0, 31.0, 30.0]
    s = [100, 90, 80, 70, 60, 50, 40]
    space = list(zip(q, s))
    assert select(space, 2.0, 85 * 10.0, 10.0) == 2   # fits from level 2
    assert select(space, 2.0, 70 * 10.0, 10.0) == 3   # last level before the cliff
    # nothing before the cliff fits: the algorithm falls through to the cliff
    assert select(space, 2.0, 65 * 10.0, 10.0) == 4


def test_beta_controls_the_cliff(select):
    q = [40.0, 39.0, 37.5, 36.0]  # drops -1, -1.5, -1.5
    s = [100, 80, 60, 40]
    space = list(zip(q, s))
    assert select(space, 2.0, 40.0, 1.0) == 3       # 1.5 < 2: no cliff
    assert select(space, 1.2, 40.0, 1.0) == 2       # 1.5 > 1.2: cliff at 2


def test_equal_first_qualities_reading(select):
    space = [(40.0, 100), (40.0, 90), (38.0, 80), (37.0, 70)]
    # previous drop 0 then a nonzero drop counts as a cliff (reading)
    assert select(space, 2.0, 75.0, 1.0) == 2
    assert select(space, 2.0, 95.0, 1.0) == 1


def test_binary_search_equals_linear_scan_on_random_monotone_tables(select):
    rng = np.random.default_rng(0)
    for _ in range(200):
        L = int(rng.integers(3, 12))
        drops = -np.abs(rng.normal(1.0, 0.2, size=L - 1))
        q = np.concatenate([[40.0], 40.0 + np.cumsum(drops)])
        s = np.sort(rng.integers(1, 1000, size=L))[::-1]
        space = list(zip(q.tolist(), s.tolist()))
        C = float(rng.integers(0, 1100))
        p = select(space, 10.0, C, 1.0)   # beta 10: no cliff here
        exp = lowest_fitting(space, range(L), C)
        assert p == (exp if exp is not None else L - 1)


def test_usage_keep_mask_drops_least_used_with_id_ties(keep_mask):
    usage = np.array([5, 0, 3, 0, 9, 3, 1], dtype=np.int64)
    m = keep_mask(usage, 7, 3, 3, 0.5)   # floor(3.5) = 3 dropped
    flat = m.reshape(-1)
    assert list(flat[:7]) == [1, 0, 1, 0, 1, 1, 0]     # ids 1, 3 (usage 0), 6 (usage 1)
    assert list(flat[7:]) == [0, 0]
    assert keep_mask(usage, 7, 3, 3, 0.0).reshape(-1)[:7].all()
    assert not keep_mask(usage, 7, 3, 3, 1.0).reshape(-1).any()
    m2 = keep_mask(usage, 7, 3, 3, 0.3)  # floor(2.1) = 2: the two zeros
    assert list(m2.reshape(-1)[:7]) == [1, 0, 1, 0, 1, 1, 1]


def test_product_selection_equals_oracle_on_random_tables():
    """Random tables with cliffs, flat stretches and equal sizes."""
    rng = np.random.default_rng(1)
    for _ in range(2000):
        L = int(rng.integers(1, 12))
        drops = -np.abs(rng.normal(1.0, 0.6, size=L - 1))
        drops[rng.random(L - 1) < 0.15] = 0.0
        drops[rng.random(L - 1) < 0.1] *= 6.0
        q = np.concatenate([[35.0], 35.0 + np.cumsum(drops)])
        s = np.sort(rng.integers(1, 50, size=L))[::-1] * 10
        space = list(zip(q.tolist(), s.tolist()))
        beta = float(rng.choice([1.5, 2.0, 4.0]))
        C = float(rng.integers(0, 520))
        assert prune.select_level(space, beta, C, 1.0) == oracle.select_level(space, beta, C, 1.0)


def test_product_keep_masks_equal_oracle_on_random_usage():
    rng = np.random.default_rng(2)
    n, gw, gh = 500, 23, 22
    usage = rng.integers(0, 6, n)
    for level in np.linspace(0.0, 1.0, 11):
        np.testing.assert_array_equal(prune.usage_keep_mask(usage, n, gw, gh, level),
                                      oracle.usage_keep_mask(usage, n, gw, gh, level))
