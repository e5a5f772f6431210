"""Pins of the median-cut palette oracle (Sec. 4.1 compression; Heckbert's median cut).

A hand-worked example, the one-dimensional case (median cut in 1-D is equal-count
quantisation of the sorted values), refinement and error monotonicity across
rounds, tie rules and box sizes.  None of these calls the HIP library.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import palette as P


def test_hand_worked_six_points():
    # widths (10, 9): split on x at the median -> {0, 2, 4} | {5, 3, 1};
    # then {0, 2, 4} is widest in y (9 > 4) -> {0} | {2, 4};
    #      {1, 3, 5} is widest in x (4 > 2) -> {5} | {3, 1}
    X = np.array([[0, 0], [10, 1], [2, 5], [8, 2], [4, 9], [6, 3]], float)
    idx, pal, cnt = P.median_cut(X, 1)
    assert idx.tolist() == [0, 1, 0, 1, 0, 1]
    np.testing.assert_allclose(pal, [[2, 14 / 3], [8, 2]], rtol=1e-15)
    idx, pal, cnt = P.median_cut(X, 2)
    assert idx.tolist() == [0, 3, 1, 3, 1, 2]
    assert cnt.tolist() == [1, 2, 1, 2]
    np.testing.assert_allclose(pal, [[0, 0], [3, 7], [6, 3], [9, 1.5]], rtol=1e-15)


def _halving_sizes(n, bits):
    sizes = [n]
    for _ in range(bits):
        sizes = [s for x in sizes for s in (x // 2, x - x // 2)]
    return sizes


@pytest.mark.parametrize("n,bits", [(1000, 4), (37, 3), (5, 4)])
def test_one_dimension_is_equal_count_quantiles(n, bits):
    rng = np.random.default_rng(n)
    x = rng.normal(size=n)
    x[::7] = x[0]                                   # ties, resolved by leaf index
    idx, pal, cnt = P.median_cut(x[:, None], bits)
    order = np.lexsort((np.arange(n), x))
    boxes = idx[order]
    assert np.all(np.diff(boxes) >= 0)              # consecutive groups of the sorted values
    assert cnt.tolist() == _halving_sizes(n, bits)
    for b in range(2 ** bits):
        if cnt[b]:
            assert pal[b, 0] == pytest.approx(x[idx == b].mean(), rel=1e-14, abs=1e-15)
        else:
            assert pal[b, 0] == 0.0


def test_rounds_refine_and_error_never_grows():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(3000, 12)) * rng.uniform(0.1, 2.0, size=12)
    prev_idx, prev_err = None, None
    for bits in range(0, 9):
        idx, pal, cnt = P.median_cut(X, bits)
        err = float(((X - pal[idx]) ** 2).sum())
        assert sorted(set(cnt.tolist())) == sorted(set(_halving_sizes(3000, bits)))
        if prev_idx is not None:
            assert np.array_equal(idx // 2, prev_idx)   # every box of round r is split in round r + 1
            assert err <= prev_err * (1 + 1e-12)
        prev_idx, prev_err = idx, err


def test_ties_and_signed_zeros():
    X = np.zeros((8, 3))
    X[1::2, 0] = -0.0
    idx, _, _ = P.median_cut(X, 2)
    assert idx.tolist() == [0, 0, 1, 1, 2, 2, 3, 3]   # identical rows: split by leaf index
    # equal widths: the lowest dimension is cut
    idx, _, _ = P.median_cut(np.array([[0.0, 1.0], [1.0, 0.0]]), 1)
    assert idx.tolist() == [0, 1]
    # a box with one member leaves its lower sibling empty
    idx, pal, cnt = P.median_cut(np.array([[1.0], [2.0]]), 2)
    assert cnt.tolist() == [0, 1, 0, 1] and idx.tolist() == [1, 3]
    assert np.all(pal[[0, 2]] == 0.0)


def test_quantize_tree_decodes_through_the_palette():
    rng = np.random.default_rng(5)
    sh = rng.normal(size=(500, 3, 4)).astype(np.float32)
    sig = rng.uniform(-1, 5, size=500)
    s16, idx, pal, dec = P.quantize_tree(sig, sh, 5)
    np.testing.assert_array_equal(s16, O.round_storage(sig, "f16"))
    np.testing.assert_array_equal(dec, pal[idx])
    assert pal.shape == (32, 3, 4)
    np.testing.assert_array_equal(pal, O.round_storage(pal, "f16"))
