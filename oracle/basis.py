"""Multilevel basis W, L built explicitly, by per-cell SVD.  TEST INFRASTRUCTURE.

Paper, Sec. 3.1 (multilevel basis construction), followed step by step
with dense N-vectors:

  * start at the deepest level; a leaf cell with s points carries the s
    unit vectors e_i of its points as candidates;
  * for each cell form M = X^T V (p x m), V the N x m matrix of the
    candidate vectors, and take the SVD M = U D V'^T;  the first a right
    singular vectors (a = number of nonzero singular values) combine the
    candidates into scaling vectors phi, the remaining m - a into
    wavelets psi, which are orthogonal to the columns of X;
  * a parent cell takes the union of its two children's scaling vectors
    as candidates and repeats the step; the root's scaling vectors span
    the column space of X and form L (p x N);
  * W stacks the wavelet rows level by level, finest first:
    W = [W_t; ...; W_0] ((N - p) x N); P = [W; L] is orthogonal.

Readings:  "nonzero" singular value means sigma_i > rank_rtol * sigma_1
(rank_rtol = 1e-10); within a level, cells are in preorder; within a
cell, wavelets follow the singular-vector order.  X uses raw
coordinates (oracle.design).  W is not unique (tree ties, SVD signs and
rotations inside a cell); only basis-independent quantities are ever
compared with another implementation.

Pins (tests/test_oracle_basis.py): P P^T = I, W X = 0, the direct-sum
dimension count, the per-level counts of the paper's sparsity table
(fixture tests/golden/tabsparse_size.txt, reproduced by `level_sizes`),
support of every wavelet inside its cell, and the condition-number
inequality kappa(W C W^T) <= kappa(C) (Proposition in Sec. 3).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .design import design_matrix
from .kdtree import KdTree


class RankError(RuntimeError):
    pass


@dataclass
class Basis:
    W: np.ndarray          # (N - p, N), columns indexed by INPUT point index
    L: np.ndarray          # (p, N)
    level_rows: dict       # level q -> number of wavelet rows
    node_rows: dict        # node -> (row offset in W, count)
    node_a: dict           # node -> number of scaling vectors
    p: int


def build_basis(points: np.ndarray, tree: KdTree, w: int, rank_rtol: float = 1e-10) -> Basis:
    pts = np.asarray(points, dtype=np.float64)
    n = pts.shape[0]
    X = design_matrix(pts, w)
    p = X.shape[1]
    scaling = {}           # node -> N x a matrix of scaling vectors
    wavelets = {}          # node -> N x (m - a)
    node_a = {}

    # children before parents: decreasing depth
    order = sorted(range(tree.n_nodes), key=lambda v: -tree.depth[v])
    for v in order:
        if tree.is_leaf(v):
            idx = tree.perm[tree.begin[v]:tree.end[v]]
            cand = np.zeros((n, idx.size))
            cand[idx, np.arange(idx.size)] = 1.0
        else:
            cand = np.concatenate([scaling.pop(tree.left[v]), scaling.pop(tree.right[v])], axis=1)
        M = X.T @ cand                              # p x m
        _, sv, vh = np.linalg.svd(M, full_matrices=True)
        vfull = vh.T                                # m x m, columns = right singular vectors
        a = int(np.sum(sv > rank_rtol * sv[0])) if sv.size and sv[0] > 0 else 0
        scaling[v] = cand @ vfull[:, :a]
        wavelets[v] = cand @ vfull[:, a:]
        node_a[v] = a

    root = 0
    if node_a[root] != p:
        raise RankError(f"root scaling rank {node_a[root]} < p = {p}")
    L = scaling[root].T
    rows, level_rows, node_rows = [], {}, {}
    off = 0
    for q in range(tree.max_depth, -1, -1):
        level_rows[q] = 0
        for v in range(tree.n_nodes):                # preorder within the level
            if tree.depth[v] != q:
                continue
            wv = wavelets[v].T
            node_rows[v] = (off, wv.shape[0])
            off += wv.shape[0]
            level_rows[q] += wv.shape[0]
            rows.append(wv)
    W = np.concatenate(rows, axis=0) if rows else np.zeros((0, n))
    return Basis(W=W, L=L, level_rows=level_rows, node_rows=node_rows, node_a=node_a, p=p)


def level_sizes(n: int, t: int, p: int) -> list[int]:
    """Count-only form of the construction for a complete tree of depth t
    over n points (cells split by rank, ceil(m/2) to the left) on generic
    data, where every M has full rank: a cell with m candidates keeps
    a = min(m, p) scaling vectors and emits m - a wavelets.  Returns the
    number of wavelets at levels q = 0..t."""
    sizes = [n]
    for _ in range(t):
        sizes = [s for m in sizes for s in ((m + 1) // 2, m // 2)]
    counts = [0] * (t + 1)
    carry = sizes                                   # candidates of the level-t cells
    for q in range(t, -1, -1):
        nxt = []
        for m in carry:
            a = min(m, p)
            counts[q] += m - a
            nxt.append(a)
        carry = [nxt[i] + nxt[i + 1] for i in range(0, len(nxt) - 1, 2)]
    return counts
