"""Host C++ kd-tree and multilevel basis, called through the C ABI on the
CPU, against the oracle: the tree bit-exact, the basis by basis-independent
invariants (orthogonality, vanishing moments, per-level counts, per-level
projectors), and the error paths."""
import math

import numpy as np
import pytest

import synth
from oracle.basis import build_basis as oracle_basis
from oracle.design import design_matrix
from oracle.kdtree import build_kdtree
from paper_1701_00285_amd import Basis, MlblupError, Tree


CASES = [(1000, 2, 1, 32), (700, 3, 2, 64), (513, 5, 1, 20), (300, 2, 2, 7), (257, 10, 1, 30)]


@pytest.mark.parametrize("n,d,w,leaf", CASES)
def test_tree_matches_oracle_exactly(n, d, w, leaf):
    pts = synth.uniform_cloud(n, d, seed=100 + n)
    t = Tree(pts, leaf)
    o = build_kdtree(pts, leaf)
    np.testing.assert_array_equal(t.perm, o.perm)
    nd = t.nodes()
    assert t.n_nodes == o.n_nodes and t.max_depth == o.max_depth
    np.testing.assert_array_equal(nd["begin"], o.begin)
    np.testing.assert_array_equal(nd["end"], o.end)
    np.testing.assert_array_equal(nd["depth"], o.depth)
    np.testing.assert_array_equal(nd["axis"], o.axis)
    np.testing.assert_array_equal(nd["left"], o.left)
    np.testing.assert_array_equal(nd["right"], o.right)
    np.testing.assert_array_equal(nd["threshold"], o.threshold)


def test_tree_workload_clusters_matches_oracle():
    wl = synth.make_config(3, n=4000, n_targets=10, with_z=False)
    t = Tree(wl.points, 64)
    o = build_kdtree(wl.points, 64)
    np.testing.assert_array_equal(t.perm, o.perm)


def _projector(rows):
    return rows.T @ rows


@pytest.mark.parametrize("n,d,w,leaf", CASES)
def test_basis_invariants_and_oracle_subspaces(n, d, w, leaf):
    pts = synth.uniform_cloud(n, d, seed=100 + n)
    t = Tree(pts, leaf)
    b = Basis(t, w)
    p = math.comb(d + w, w)
    assert b.p == p and b.n_minus_p == n - p
    W, Lm = b.dense()
    P = np.vstack([W, Lm])
    np.testing.assert_allclose(P @ P.T, np.eye(n), atol=1e-12)
    X = design_matrix(pts[t.perm], w)
    np.testing.assert_allclose(W @ X, 0.0, atol=1e-11 * np.abs(X).max() * math.sqrt(n))
    # against the oracle's SVD basis: same per-level counts and, level by
    # level, the same subspace (projectors agree; columns map tree -> input order)
    o = build_kdtree(pts, leaf)
    ob = oracle_basis(pts, o, w)
    counts = b.level_counts()
    assert [ob.level_rows[q] for q in range(len(counts))] == list(counts)
    inv = np.empty(n, dtype=np.int64)
    inv[t.perm] = np.arange(n)
    off_c, off_o = 0, 0
    for q in range(len(counts) - 1, -1, -1):
        c = counts[q]
        Wc = W[off_c:off_c + c][:, inv]          # back to input order
        Wo = ob.W[off_o:off_o + c]
        np.testing.assert_allclose(_projector(Wc), _projector(Wo), atol=1e-10)
        off_c += c
        off_o += c
    np.testing.assert_allclose(_projector(Lm[:, inv]), _projector(ob.L), atol=1e-10)


def test_basis_level_counts_complete_tree():
    from oracle.basis import level_sizes
    pts = synth.uniform_cloud(4096, 3, seed=9)
    t = Tree(pts, 64)
    b = Basis(t, 2)
    assert list(b.level_counts()) == level_sizes(4096, t.max_depth, b.p)


def test_transform_bytes_count_every_block_once():
    """Algorithmic bytes of one transform: every cell's block read once in
    its compact WY form, K = min(m, p) reflectors of length m and the K x K
    triangle, 8 sum (K m + K^2) over the cells (a leaf's m is its point
    count, an internal cell's the sum of its children's scaling counts,
    a = min(m, p) for generic points) + 16 N."""
    pts = synth.uniform_cloud(3000, 3, seed=10)
    t = Tree(pts, 40)
    b = Basis(t, 2)
    nd = t.nodes()
    begin, end, left, right = nd["begin"], nd["end"], nd["left"], nd["right"]

    def walk(v):
        if left[v] < 0:
            m = int(end[v] - begin[v])
            k = min(m, b.p)
            return k, k * m + k * k
        al, sl = walk(left[v])
        ar, sr = walk(right[v])
        m = al + ar
        k = min(m, b.p)
        return k, k * m + k * k + sl + sr

    _, s = walk(0)
    assert b.transform_bytes() == 8 * s + 16 * 3000


def test_rank_error_collinear_quadratic():
    pts = np.zeros((40, 2))
    pts[:, 0] = np.linspace(0, 1, 40)
    t = Tree(pts, 8)
    with pytest.raises(MlblupError, match="ERANK"):
        Basis(t, 2)


def test_rank_error_duplicates():
    pts = np.repeat(synth.uniform_cloud(3, 2, 1), 20, axis=0)   # 3 distinct sites, linear trend OK, quadratic not
    t = Tree(pts, 8)
    Basis(t, 1)
    with pytest.raises(MlblupError, match="ERANK"):
        Basis(t, 2)


def test_invalid_arguments():
    with pytest.raises(MlblupError, match="EINVAL"):
        Tree(np.zeros((0, 2)), 8)
    bad = synth.uniform_cloud(10, 2, 1)
    bad[3, 1] = np.nan
    with pytest.raises(MlblupError, match="EINVAL"):
        Tree(bad, 4)
    t = Tree(synth.uniform_cloud(5, 2, 1), 2)
    with pytest.raises(MlblupError, match="EINVAL"):
        Basis(t, 2)        # N = 5 <= p = 6
    with pytest.raises(MlblupError, match="EINVAL"):
        Basis(t, 40)


def test_large_workload_basis_builds():
    wl = synth.make_config(2, n=65536, n_targets=1, with_z=False)
    t = Tree(wl.points, wl.leaf_max)
    b = Basis(t, wl.degree_w)
    assert t.max_depth == 10 and b.n_minus_p == 65536 - 10
    assert sum(b.level_counts()) == 65536 - 10


def test_loglik_workspace_counts_the_partial_transform_rows():
    """Rows of [W_t; ...; W_n] = wavelets at levels >= n; the workspace holds
    the N x N covariance and the N~ x N first analysis; level outside
    [0, levels) is rejected."""
    import ctypes as C
    from paper_1701_00285_amd import _lib as L
    pts = synth.uniform_cloud(1500, 2, seed=11)
    t = Tree(pts, 32)
    b = Basis(t, 1)
    counts = b.level_counts()
    for level in range(b.levels):
        by, rows = C.c_int64(), C.c_int64()
        assert L.lib().mlblup_loglik_workspace_bytes(b.h, level, C.byref(by), C.byref(rows)) == L.OK
        assert rows.value == int(counts[level:].sum())
        assert by.value >= 8 * (1500 * 1500 + rows.value * 1500)
    by = C.c_int64()
    assert L.lib().mlblup_loglik_workspace_bytes(b.h, b.levels, C.byref(by), None) == L.EINVAL
    assert L.lib().mlblup_loglik_workspace_bytes(b.h, -1, C.byref(by), None) == L.EINVAL


def test_precond_workspace_by_kind():
    """The coarse kind needs the N x N covariance besides the cell-block
    build; the other kinds need what the plain query gives."""
    import ctypes as C
    from paper_1701_00285_amd import PREC_BLOCK, PREC_COARSE, PREC_JACOBI
    from paper_1701_00285_amd import _lib as L
    pts = synth.uniform_cloud(3000, 3, seed=12)
    b = Basis(Tree(pts, 64), 2)
    plain, by = C.c_int64(), C.c_int64()
    assert L.lib().mlblup_precond_workspace_bytes(b.h, C.byref(plain)) == L.OK
    for kind in (PREC_JACOBI, PREC_BLOCK):
        assert L.lib().mlblup_precond_workspace_bytes_kind(b.h, kind, C.byref(by)) == L.OK
        assert by.value == plain.value
    assert L.lib().mlblup_precond_workspace_bytes_kind(b.h, PREC_COARSE, C.byref(by)) == L.OK
    counts = b.level_counts()
    nc = int(counts[:-1].sum())
    assert by.value >= 8 * (3000 * 3000 + nc * 3000) and by.value >= plain.value
