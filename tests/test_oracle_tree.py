"""Pins for the oracle's cluster tree and block list (no GPU)."""
import numpy as np
import pytest

from oracle import tree as T


def test_hand_example_n7():
    nb = T.node_bounds(7, 2)
    assert nb == [[0, 7], [0, 4, 7], [0, 2, 4, 6, 7]]


@pytest.mark.parametrize("n,leaf,depth", [(2048, 128, 4), (65536, 256, 8), (262144, 512, 9),
                                          (1 << 20, 256, 12), (1, 1, 0), (5, 2, 2), (3, 4, 0),
                                          (2000, 8, 8)])
def test_depth_for_leaf(n, leaf, depth):
    assert T.depth_for_leaf(n, leaf) == depth
    sizes = np.diff(T.node_bounds(n, depth)[depth])
    assert sizes.max() <= leaf
    if depth:
        assert np.diff(T.node_bounds(n, depth - 1)[depth - 1]).max() > leaf


def test_uniform_leaves_2048():
    assert set(np.diff(T.node_bounds(2048, 4)[4])) == {128}


@pytest.mark.parametrize("n", [1, 2, 3, 7, 100, 1000, 2047, 4097])
def test_level_sizes_floor_ceil_and_nesting(n):
    depth = 6
    nb = T.node_bounds(n, depth)
    for k in range(depth + 1):
        b = np.array(nb[k])
        assert b[0] == 0 and b[-1] == n and len(b) == (1 << k) + 1
        sz = np.diff(b)
        assert set(sz) <= {n // (1 << k), -(-n // (1 << k))}
        if k:
            # every parent boundary is a child boundary, left child >= right child
            assert np.array_equal(b[::2], np.array(nb[k - 1]))
            assert np.all(sz[0::2] >= sz[1::2])


@pytest.mark.parametrize("n,depth", [(7, 2), (64, 3), (100, 4), (33, 5), (1, 3)])
def test_blocks_and_leaves_tile_the_matrix_once(n, depth):
    """Eq. (2.1) applied recursively: leaves plus off-diagonal blocks cover
    every (i, j) exactly once."""
    cover = np.zeros((n, n), dtype=int)
    for a, m in T.leaves(n, depth):
        cover[a:a + m, a:a + m] += 1
    blks = T.blocks(n, depth)
    assert len(blks) == (1 << (depth + 1)) - 2
    for b in blks:
        cover[b.row0:b.row0 + b.nrows, b.col0:b.col0 + b.ncols] += 1
    assert np.all(cover == 1)


def test_canonical_order_upper_before_lower():
    blks = T.blocks(100, 3)
    for i, b in enumerate(blks):
        assert b.index == i
        assert b.index == (1 << b.level) - 2 + b.row_node
        assert b.col_node == b.row_node ^ 1
    # within a sibling pair, the upper block lies above the diagonal
    for b in blks:
        if b.upper:
            assert b.row0 + b.nrows <= b.col0
        else:
            assert b.col0 + b.ncols <= b.row0
    levels = [b.level for b in blks]
    assert levels == sorted(levels)


def test_given_leaf_bounds_with_empty_nodes():
    lb = [0, 0, 3, 3, 5]
    nb = T.node_bounds(5, 2, lb)
    assert nb == [[0, 5], [0, 3, 5], [0, 0, 3, 3, 5]]
    blks = T.blocks(5, 2, lb)
    assert blks[2].nrows == 0 and blks[3].ncols == 0
    with pytest.raises(ValueError):
        T.node_bounds(5, 2, [0, 3, 2, 4, 5])
