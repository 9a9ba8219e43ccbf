"""kd-tree domain decomposition.  TEST INFRASTRUCTURE.

Paper, Sec. 3.1: the cell-split rule (algorithm "Rule for cell-split")
picks the coordinate axis along which the cell's points have maximal
variance, projects the points on it and splits at the median;
"InitialTree" starts at node 0 / depth 0 and "MakeTree" numbers the
nodes in preorder (left subtree first), recursing until a cell is small
enough to be a leaf.

Readings where the paper is silent or ambiguous:
  * leaf iff the cell holds at most n0 points (the listing says "< n0",
    the text says a leaf holds a maximum number of observations);
  * the rule uses the cell's own points (the listing passes the full set);
  * median split by rank: points are ordered by (projection, input
    index) and the first ceil(m/2) go left; threshold = largest left
    projection, so "x . v <= threshold goes left" holds for every point
    except ties across the split, which the rank order settles;
  * equal variances: the lowest axis index wins;
  * inside a leaf the points are listed by increasing input index.
Any valid tree gives the same BLUP; these readings only make the tree
deterministic so that two implementations can be compared exactly.

Pins (tests/test_oracle_tree.py): brute-force checks of every node
(axis is the arg-max of the variances, left/right partition by rank,
sizes differ by at most one, every leaf holds <= n0 points, every
internal node > n0), perm is a permutation, preorder numbering.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class KdTree:
    n: int
    d: int
    leaf_max: int
    perm: np.ndarray                      # tree position -> input index
    begin: list = field(default_factory=list)
    end: list = field(default_factory=list)
    depth: list = field(default_factory=list)
    axis: list = field(default_factory=list)
    threshold: list = field(default_factory=list)
    left: list = field(default_factory=list)
    right: list = field(default_factory=list)

    @property
    def n_nodes(self) -> int:
        return len(self.begin)

    @property
    def max_depth(self) -> int:
        return max(self.depth)

    def is_leaf(self, v: int) -> bool:
        return self.left[v] < 0


def build_kdtree(points: np.ndarray, leaf_max: int) -> KdTree:
    pts = np.asarray(points, dtype=np.float64)
    n, d = pts.shape
    tree = KdTree(n=n, d=d, leaf_max=leaf_max, perm=np.zeros(n, dtype=np.int64))

    def make(idx: np.ndarray, depth: int, start: int) -> int:
        node = tree.n_nodes
        tree.begin.append(start)
        tree.end.append(start + idx.size)
        tree.depth.append(depth)
        tree.axis.append(-1)
        tree.threshold.append(0.0)
        tree.left.append(-1)
        tree.right.append(-1)
        if idx.size <= leaf_max:
            tree.perm[start:start + idx.size] = np.sort(idx)
            return node
        vrs = pts[idx].var(axis=0)
        ax = int(np.argmax(vrs))
        proj = pts[idx, ax]
        order = np.lexsort((idx, proj))          # by projection, then input index
        n_left = (idx.size + 1) // 2
        li, ri = idx[order[:n_left]], idx[order[n_left:]]
        tree.axis[node] = ax
        tree.threshold[node] = float(proj[order[n_left - 1]])
        tree.left[node] = make(li, depth + 1, start)
        tree.right[node] = make(ri, depth + 1, start + n_left)
        return node

    make(np.arange(n, dtype=np.int64), 0, 0)
    return tree
