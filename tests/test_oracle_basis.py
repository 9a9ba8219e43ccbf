"""Pins for oracle.basis: orthogonality, vanishing moments, direct-sum
count, the paper's per-level counts (sparsity table "Size" column),
locality, the condition-number inequality, and planted mistakes."""
import numpy as np
import pytest

import synth
from conftest import golden
from oracle import basis as B
from oracle.design import design_matrix
from oracle.kdtree import build_kdtree
from oracle.matern import cov_matrix


def _setup(n, d, w, leaf, seed=0):
    pts = synth.uniform_cloud(n, d, seed)
    tree = build_kdtree(pts, leaf)
    return pts, tree, B.build_basis(pts, tree, w)


@pytest.mark.parametrize("n,d,w,leaf", [(200, 2, 1, 8), (300, 2, 2, 16), (257, 3, 2, 20), (150, 5, 1, 12)])
def test_orthogonal_and_vanishing_moments(n, d, w, leaf):
    pts, tree, bas = _setup(n, d, w, leaf)
    X = design_matrix(pts, w)
    P = np.vstack([bas.W, bas.L])
    assert P.shape == (n, n)
    np.testing.assert_allclose(P @ P.T, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(bas.W @ X, 0, atol=1e-11 * np.abs(X).max())
    # rows of L span col(X): projecting X onto them reproduces X
    np.testing.assert_allclose(bas.L.T @ (bas.L @ X), X, atol=1e-11 * np.abs(X).max())
    assert bas.W.shape[0] == n - bas.p


def test_wavelets_supported_in_their_cell():
    pts, tree, bas = _setup(300, 2, 2, 16)
    for v, (off, cnt) in bas.node_rows.items():
        inside = np.zeros(300, dtype=bool)
        inside[tree.perm[tree.begin[v]:tree.end[v]]] = True
        assert np.all(np.abs(bas.W[off:off + cnt][:, ~inside]) < 1e-13)


def test_counts_complete_tree():
    n, d, w, leaf = 512, 3, 1, 16       # p = 4, complete tree of depth 5
    pts, tree, bas = _setup(n, d, w, leaf)
    t = tree.max_depth
    counts = B.level_sizes(n, t, bas.p)
    assert [bas.level_rows[q] for q in range(t + 1)] == counts
    assert sum(counts) == n - bas.p


def test_paper_sparsity_table_sizes():
    """Cumulative wavelet counts at levels t..i equal the table's Size column."""
    for N, t, i, size in golden("tabsparse_size.txt"):
        counts = B.level_sizes(N, t, 1001)
        assert sum(counts[i:]) == size


def test_level_bound_lemma():
    """Lemma (Sec. 3.1): with n0 < 2p, level q holds at most p 2^q vectors."""
    pts, tree, bas = _setup(600, 2, 2, 10)     # p = 6, n0 = 10 < 12
    for q, c in bas.level_rows.items():
        assert c <= bas.p * 2 ** q


def test_condition_number_inequality():
    pts, tree, bas = _setup(250, 2, 2, 16)
    C = cov_matrix(pts, pts, 1.5, 0.3)
    CW = bas.W @ C @ bas.W.T
    ev = np.linalg.eigvalsh(C)
    evw = np.linalg.eigvalsh(CW)
    assert evw.min() >= ev.min() * (1 - 1e-9) and evw.max() <= ev.max() * (1 + 1e-9)
    assert evw.max() / evw.min() <= ev.max() / ev.min()


def test_rank_error_for_degenerate_points():
    pts = np.zeros((30, 2))
    pts[:, 0] = np.linspace(0, 1, 30)         # collinear: quadratic trend rank < p
    tree = build_kdtree(pts, 8)
    with pytest.raises(B.RankError):
        B.build_basis(pts, tree, 2)


def test_planted_mistake_swapped_singular_vectors(monkeypatch):
    """Taking the wavelets from the leading right singular vectors (a swap
    of the two blocks) must break the vanishing-moment pin."""
    real_svd = np.linalg.svd

    def swapped(M, full_matrices=True):
        u, s, vh = real_svd(M, full_matrices=full_matrices)
        return u, s, vh[::-1]
    monkeypatch.setattr(B.np.linalg, "svd", swapped)
    pts = synth.uniform_cloud(120, 2, 5)
    tree = build_kdtree(pts, 12)
    try:
        bas = B.build_basis(pts, tree, 1)
    except B.RankError:
        return
    X = design_matrix(pts, 1)
    assert np.abs(bas.W @ X).max() > 1e-6
