"""Pins for the row-major triangle index map (Section 4.2, "Row & Column")."""
import math

import pytest

from oracle import index_map as im


def test_n4_example():
    # the row-major traversal of Section 4.1 for n = 4
    assert list(im.enumerate_pairs(4)) == [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    assert [im.pair_of_index(4, k) for k in range(6)] == list(im.enumerate_pairs(4))
    # S_0 = n-1, S_1 = S_0 + (n-2), ..., S_{n-1} = number of edges
    assert im.S(4, 0) == 3 and im.S(4, 1) == 5 and im.S(4, 3) == 6


@pytest.mark.parametrize("n", [2, 3, 5, 17, 64, 257, 1000])
def test_exhaustive_forward_and_inverse(n):
    for k, (r, c) in enumerate(im.enumerate_pairs(n)):
        assert im.pair_index(n, r, c) == k
        assert im.pair_of_index(n, k) == (r, c)
    assert im.num_pairs(n) == im.S(n, n - 1) == n * (n - 1) // 2


def test_edge_counts():
    assert im.num_pairs(2000) == 1_999_000
    assert im.num_pairs(50_000) == 1_249_975_000
    assert im.num_pairs(600_000) == 179_999_700_000          # ~1.8e11 (Section 1)
    assert im.num_pairs(100_000) == 4_999_950_000            # 4.66 GiB at one byte per edge
    assert round(4_999_950_000 / 2**30, 2) == 4.66
    assert im.num_pairs(0) == 0 and im.num_pairs(1) == 0


def test_capacity_formula():
    for n in (2, 10, 107_000, 600_000):
        assert im.capacity_words(im.num_pairs(n)) == pytest.approx(n, abs=1e-6 * n)


def test_paper_inverse_at_600k_row_boundaries():
    """The float64 closed form stays exact at n = 600,000 on and around row starts."""
    n = 600_000
    rows = list(range(0, 50)) + list(range(n - 60, n - 1)) + [1000, 12345, 299_999, 300_000, 456_789]
    for r in rows:
        s = im.S(n, r - 1)
        e = im.S(n, r)
        for k in (s, s + 1, e - 2, e - 1):
            if s <= k < e:
                assert im.pair_of_index(n, k) == (r, r + 1 + k - s)
        if r > 0:
            assert im.pair_of_index(n, s - 1) == (r - 1, n - 1)
    with pytest.raises(ValueError):
        im.pair_of_index(n, im.num_pairs(n))
    assert math.isclose(im.S(n, n - 1), 1.8e11, rel_tol=1e-3)
