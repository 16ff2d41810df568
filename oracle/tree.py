"""Cluster tree and canonical block list (oracle side).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

* Def. 2.1: a complete binary tree of depth l whose level-k nodes I_1^k ..
  I_{2^k}^k partition {1..n} into consecutive (possibly empty) ranges, and
  node I_i^k has children I_{2i-1}^{k+1}, I_{2i}^{k+1}.
* Sect. 4, experimental setup: the left child takes the ceiling of half the
  parent's size, so level-k nodes have floor(n/2^k) or ceil(n/2^k) indices.
* Eq. (2.1): every diagonal block at level k-1 splits into two diagonal
  blocks and two off-diagonal blocks at level k; the upper one has the rows
  of the odd child and the columns of the even child, the lower one the
  reverse.

Indices here are 0-based: node j of level k (j = 0..2^k-1) is the paper's
I_{j+1}^k, a half-open range [bounds[k][j], bounds[k][j+1]).  The canonical
block order is level ascending, then row node ascending; within a sibling
pair the upper block (row node even) precedes the lower one.  So the block
whose rows are node j of level k has index (2^k - 2) + j and its columns
are node j XOR 1.
"""
from __future__ import annotations

from dataclasses import dataclass


def depth_for_leaf(n: int, leaf: int) -> int:
    """Smallest depth l >= 0 whose ceil-split leaves hold at most ``leaf``
    indices, i.e. the smallest l with leaf * 2^l >= n."""
    if n < 1 or leaf < 1:
        raise ValueError("n and leaf must be positive")
    depth = 0
    while leaf * (1 << depth) < n:
        depth += 1
    return depth


def node_bounds(n: int, depth: int, leaf_bounds=None) -> list[list[int]]:
    """Boundaries n_0^k <= ... <= n_{2^k}^k for k = 0..depth (Def. 2.1).

    Without ``leaf_bounds`` the tree is built top-down by the ceil split.
    With ``leaf_bounds`` (2^depth + 1 non-decreasing integers from 0 to n)
    the leaves are given and every coarser level takes every other boundary
    of the level below (a parent is the union of its two children).
    """
    if depth < 0:
        raise ValueError("depth must be >= 0")
    if leaf_bounds is None:
        levels = [[0, n]]
        for _ in range(depth):
            prev = levels[-1]
            nxt = [0]
            for j in range(len(prev) - 1):
                a, b = prev[j], prev[j + 1]
                left = (b - a + 1) // 2          # ceil((b - a) / 2)
                nxt.append(a + left)
                nxt.append(b)
            levels.append(nxt)
        return levels
    lb = [int(v) for v in leaf_bounds]
    if len(lb) != (1 << depth) + 1 or lb[0] != 0 or lb[-1] != n:
        raise ValueError("leaf_bounds must hold 2^depth + 1 values from 0 to n")
    if any(lb[i] > lb[i + 1] for i in range(len(lb) - 1)):
        raise ValueError("leaf_bounds must be non-decreasing")
    levels = []
    for k in range(depth + 1):
        step = 1 << (depth - k)
        levels.append(lb[::step])
    return levels


@dataclass(frozen=True)
class Block:
    index: int      # canonical index
    level: int      # k = 1..depth
    row_node: int   # j, 0-based; the paper's U_{j+1}^{(k)}
    col_node: int   # j ^ 1; the paper's V_{(j^1)+1}^{(k)}
    row0: int
    nrows: int
    col0: int
    ncols: int

    @property
    def upper(self) -> bool:
        return self.row_node % 2 == 0


def blocks(n: int, depth: int, leaf_bounds=None) -> list[Block]:
    """The 2^(depth+1) - 2 off-diagonal blocks in canonical order (eq. (2.1))."""
    nb = node_bounds(n, depth, leaf_bounds)
    out = []
    for k in range(1, depth + 1):
        bk = nb[k]
        for j in range(1 << k):
            c = j ^ 1
            out.append(Block(len(out), k, j, c, bk[j], bk[j + 1] - bk[j],
                             bk[c], bk[c + 1] - bk[c]))
    return out


def leaves(n: int, depth: int, leaf_bounds=None) -> list[tuple[int, int]]:
    """(start, size) of the 2^depth diagonal leaf blocks."""
    lb = node_bounds(n, depth, leaf_bounds)[depth]
    return [(lb[i], lb[i + 1] - lb[i]) for i in range(1 << depth)]
