"""Host sparsity pattern of C~^n_W (Sec. 4.1 tree search with distance
tau), called through the C ABI on the CPU, against the oracle's pattern:
bit-exact for every level and several tau, including trees with leaves at
two depths; nnz equals the pattern's sum; tau = inf keeps everything; bad
tau and level are rejected."""
import math

import numpy as np
import pytest

import synth
from oracle import likelihood as OL
from oracle.basis import build_basis as oracle_basis
from oracle.kdtree import build_kdtree
from paper_1701_00285_amd import Basis, MlblupError, Tree

# (1000, 2, 1, 31) and (700, 3, 2, 43) have leaves at two depths
CASES = [(1000, 2, 1, 32), (1000, 2, 1, 31), (700, 3, 2, 43), (513, 5, 1, 20), (300, 2, 2, 7), (257, 10, 1, 30)]


@pytest.mark.parametrize("n,d,w,leaf", CASES)
def test_pattern_matches_oracle_exactly(n, d, w, leaf):
    pts = synth.uniform_cloud(n, d, seed=100 + n)
    t = Tree(pts, leaf)
    b = Basis(t, w)
    ot = build_kdtree(pts, leaf)
    ob = oracle_basis(pts, ot, w)
    depths = set(ot.depth[v] for v in range(ot.n_nodes) if ot.is_leaf(v))
    for level in range(b.levels):
        for tau in (0.0, 0.01, 0.07, 0.25):
            nnz, m = b.sparsity_pattern(level, tau, mask=True)
            om = OL.sparsity_mask(pts, ot, ob, level, tau)
            assert m.shape == om.shape
            np.testing.assert_array_equal(m, om, err_msg=f"level {level} tau {tau} leaf depths {depths}")
            assert nnz == int(om.sum())
        nt = m.shape[0]
        assert b.sparsity_pattern(level, math.inf) == nt * nt


def test_pattern_thins_out_with_small_tau():
    pts = synth.uniform_cloud(4000, 2, seed=3)
    b = Basis(Tree(pts, 32), 1)
    nt = int(b.level_counts().sum())
    frac = [b.sparsity_pattern(0, tau) / nt**2 for tau in (0.0, 0.02, 0.1, 0.5, 2.0)]
    assert all(x <= y for x, y in zip(frac, frac[1:]))
    assert frac[0] < 0.2 and frac[-1] == 1.0


def test_pattern_error_paths():
    pts = synth.uniform_cloud(300, 2, seed=4)
    b = Basis(Tree(pts, 16), 1)
    for tau in (-1e-3, float("nan")):
        with pytest.raises(MlblupError, match="EINVAL"):
            b.sparsity_pattern(0, tau)
    with pytest.raises(MlblupError, match="EINVAL"):
        b.sparsity_pattern(b.levels, 0.1)
