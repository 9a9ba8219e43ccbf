"""Pins for oracle.kdtree: brute-force checks of every node."""
import numpy as np
import pytest

import synth
from oracle.kdtree import build_kdtree


def _check(tree, pts):
    n, d = pts.shape
    assert sorted(tree.perm.tolist()) == list(range(n))
    assert tree.begin[0] == 0 and tree.end[0] == n and tree.depth[0] == 0
    counter = [0]

    def walk(v, depth):
        assert v == counter[0]              # preorder numbering
        counter[0] += 1
        assert tree.depth[v] == depth
        b, e = tree.begin[v], tree.end[v]
        if tree.left[v] < 0:
            assert 0 < e - b <= tree.leaf_max
            assert list(tree.perm[b:e]) == sorted(tree.perm[b:e])
            return
        assert e - b > tree.leaf_max
        idx = tree.perm[b:e]
        var = [np.mean((pts[idx, k] - pts[idx, k].mean()) ** 2) for k in range(d)]
        assert tree.axis[v] == int(np.argmax(var))
        l, r = tree.left[v], tree.right[v]
        assert tree.begin[l] == b and tree.end[l] == tree.begin[r] and tree.end[r] == e
        nl = tree.end[l] - b
        assert nl == (e - b + 1) // 2
        ax = tree.axis[v]
        keys = sorted((pts[i, ax], i) for i in idx)
        left_set = {i for _, i in keys[:nl]}
        assert left_set == set(tree.perm[b:b + nl].tolist())
        assert tree.threshold[v] == keys[nl - 1][0]
        walk(l, depth + 1)
        walk(r, depth + 1)

    walk(0, 0)
    assert counter[0] == tree.n_nodes


@pytest.mark.parametrize("n,d,leaf", [(1, 2, 4), (5, 2, 4), (100, 2, 8), (1000, 3, 32), (777, 5, 16)])
def test_tree_structure(n, d, leaf):
    pts = synth.uniform_cloud(n, d, seed=n + d)
    _check(build_kdtree(pts, leaf), pts)


def test_tree_with_ties():
    pts = np.zeros((40, 2))
    pts[:, 0] = np.repeat(np.arange(4), 10)      # heavy ties on axis 0
    pts[:, 1] = 0.5
    t = build_kdtree(pts, 5)
    _check(t, pts)


def test_depth_of_power_of_two():
    pts = synth.uniform_cloud(1024, 3, seed=1)
    t = build_kdtree(pts, 64)
    assert t.max_depth == 4
    assert all(t.end[v] - t.begin[v] == 64 for v in range(t.n_nodes) if t.left[v] < 0)
