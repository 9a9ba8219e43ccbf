"""Multilevel log-likelihood, its sparsified form and its maximum.  TEST
INFRASTRUCTURE.

Paper, Sec. 5.1 (the reduced multilevel likelihoods): for a level n, the
partial transform W^n = [W_t; ...; W_n] (the first N~ rows of W, finest
level first) gives

    l_n(theta) = -N~/2 log(2 pi) - 1/2 log det C^n_W - 1/2 (Z^n_W)^T (C^n_W)^-1 Z^n_W,

with C^n_W = W^n C (W^n)^T and Z^n_W = W^n Z.  Sec. 6.1 takes the
determinant and the quadratic form from one Cholesky factor G of C^n_W:
log det = 2 sum log G_ii and the quadratic form is |G^-1 Z^n_W|^2.  Here
C^n_W is formed densely from the oracle's explicit W (per-cell SVD,
oracle.basis).

Sparsified form (Sec. 4.1, algorithms SearchTree, LocalSearchTree,
ChooseLeftRule / ChooseRightRule and the block construction): the entry
psi_k^T C psi_l of two wavelets of the cells B_a (level i) and B_b (level
j >= i) is kept when the tree search from B_a with distance tau reaches B_b
at depth j; every other entry of C~^n_W is zero.  The search starts at the
root; at a node of depth j it reports the node, at a leaf above depth j it
stops, and at a split (axis k, threshold s) it enters the left subtree when
some point of B_a, moved by tau along k, can reach the side x_k <= s
(min x_k - tau <= s) and the right subtree when it can reach x_k > s
(max x_k + tau > s).  Readings: this is the hyper-rectangle rule stated in
the text (the cell's bounding box widened by tau meets the region of the
target node); the listings print the left rule with +tau and leave the
rule unused inside the recursion.  The paper computes only the blocks with
i <= j and completes the matrix by symmetry; for two cells of one level the
pair is kept when either search reaches the other.  l~_n is l_n with C~^n_W
in place of C^n_W; tau = inf keeps every entry.

The maximum over rho (nu, sigma2 fixed) is found by golden-section search
on log rho, the textbook method (Kiefer 1953): keep the two interior points
of a bracket at the golden ratio and drop the side whose interior point is
lower.

Pins (tests/test_oracle_likelihood.py): at n = 0 the determinant obeys the
restricted-likelihood identity log det(W C W^T) = log det C
+ log det(X^T C^-1 X) - log det(X^T X) (P = [W; L] orthogonal, L spanning the
columns of X), and the quadratic form equals the GLS residual form of
oracle.blup; with C = sigma2 I the value has a closed form (also after
sparsification); the condition numbers nest as the Proposition of Sec. 5.1
states; rotations of the wavelets inside a cell leave l_n unchanged; the
MLE is a local maximum.  The tree search equals the set of depth-j nodes
whose region (the box cut out by the splits on the root path) meets the
widened bounding box, checked by brute force over every node; it contains
every node holding a point inside the widened box and every descendant of
the cell; the kept set grows with tau and covers everything for tau
larger than the domain.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .basis import Basis
from .design import design_matrix
from .kdtree import KdTree
from .matern import cov_matrix

LOG_2PI = math.log(2.0 * math.pi)


def level_rows(basis: Basis, level: int) -> int:
    """N~: number of wavelet rows at levels >= level."""
    return int(sum(r for q, r in basis.level_rows.items() if q >= level))


def node_box(S, tree: KdTree, v: int):
    """(min, max) per coordinate of the points of node v."""
    P = np.asarray(S, dtype=np.float64)[tree.perm[tree.begin[v]:tree.end[v]]]
    return P.min(axis=0), P.max(axis=0)


def search_tree(tree: KdTree, lo, hi, target_depth: int, tau: float) -> list:
    """Nodes at target_depth reached from the root by the tau-widened
    bounding box [lo - tau, hi + tau] (SearchTree / LocalSearchTree)."""
    found = []

    def visit(v):
        if tree.depth[v] == target_depth:
            found.append(v)
            return
        if tree.is_leaf(v):
            return
        k, s = tree.axis[v], tree.threshold[v]
        if lo[k] - tau <= s:
            visit(tree.left[v])
        if hi[k] + tau > s:
            visit(tree.right[v])

    visit(0)
    return found


def sparsity_mask(S, tree: KdTree, basis: Basis, level: int, tau: float) -> np.ndarray:
    """Boolean N~ x N~ pattern of C~^n_W (rows in the order of basis.W)."""
    nt = level_rows(basis, level)
    cells = [v for v, (off, cnt) in basis.node_rows.items() if cnt > 0 and tree.depth[v] >= level]
    keep = {}
    for a in cells:
        lo, hi = node_box(S, tree, a)
        for j in range(tree.depth[a], tree.max_depth + 1):
            for b in search_tree(tree, lo, hi, j, tau):
                if b in basis.node_rows and basis.node_rows[b][1] > 0:
                    keep[(a, b)] = keep[(b, a)] = True
    mask = np.zeros((nt, nt), dtype=bool)
    for (a, b) in keep:
        oa, ca = basis.node_rows[a]
        ob, cb = basis.node_rows[b]
        mask[oa:oa + ca, ob:ob + cb] = True
    return mask


def multilevel_loglik(S, Z, nu, rho, basis: Basis, level: int, sigma2=1.0, tree: KdTree | None = None,
                      tau: float = math.inf):
    """(l_n, log det C^n_W, (Z^n_W)^T (C^n_W)^-1 Z^n_W, N~) for the points S
    (input order, the order of basis.W's columns) and data Z.  A finite tau
    (with the tree) evaluates the sparsified l~_n instead."""
    S = np.asarray(S, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    nt = level_rows(basis, level)
    Wn = basis.W[:nt]
    C = cov_matrix(S, S, nu, rho, sigma2)
    Cn = Wn @ C @ Wn.T
    if math.isfinite(tau):
        Cn = np.where(sparsity_mask(S, tree, basis, level, tau), Cn, 0.0)
    zn = Wn @ Z
    G = np.linalg.cholesky(Cn)
    y = sla.solve_triangular(G, zn, lower=True)
    logdet = 2.0 * float(np.sum(np.log(np.diag(G))))
    quad = float(y @ y)
    return -0.5 * (nt * LOG_2PI + logdet + quad), logdet, quad, nt


def reml_logdet(S, w, nu, rho, sigma2=1.0) -> float:
    """log det C + log det(X^T C^-1 X) - log det(X^T X): the value of
    log det(W C W^T) for any orthonormal W whose rows are orthogonal to the
    columns of X (computed without W)."""
    S = np.asarray(S, dtype=np.float64)
    X = design_matrix(S, w)
    C = cov_matrix(S, S, nu, rho, sigma2)
    cf = sla.cho_factor(C, lower=True)
    ld_c = 2.0 * float(np.sum(np.log(np.diag(cf[0]))))
    _, ld_xcx = np.linalg.slogdet(X.T @ sla.cho_solve(cf, X))
    _, ld_xx = np.linalg.slogdet(X.T @ X)
    return ld_c + float(ld_xcx) - float(ld_xx)


def golden_max(f, lo: float, hi: float, tol: float):
    """Maximum of a unimodal f on [lo, hi] by golden-section search, stopped
    when the bracket is narrower than tol; returns (x, f(x), evaluations)."""
    g = (math.sqrt(5.0) - 1.0) / 2.0
    a, b = lo, hi
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = f(c), f(d)
    evals = 2
    while b - a > tol:
        if fc >= fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = f(d)
        evals += 1
    x = 0.5 * (a + b)
    return x, f(x), evals + 1


def mle_rho(S, Z, nu, basis: Basis, level: int, rho_lo: float, rho_hi: float, log_tol: float = 1e-6,
            sigma2=1.0, tree: KdTree | None = None, tau: float = math.inf):
    """rho maximising l_level (golden section on log rho): (rho, l, evaluations)."""
    def f(lr):
        return multilevel_loglik(S, Z, nu, math.exp(lr), basis, level, sigma2, tree, tau)[0]

    lr, val, evals = golden_max(f, math.log(rho_lo), math.log(rho_hi), log_tol)
    return math.exp(lr), val, evals


def mle_nu_rho(S, Z, basis: Basis, level: int, nu_lo: float, nu_hi: float, rho_lo: float, rho_hi: float,
               nu_tol: float = 1e-3, log_rho_tol: float = 1e-4, sigma2=1.0, tree: KdTree | None = None,
               tau: float = math.inf):
    """(nu, rho) maximising l_level by the profile likelihood: golden
    section over nu, each point the golden-section rho maximum.  Returns
    (nu, rho, l)."""
    best = {}

    def profile(nu):
        rho, val, _ = mle_rho(S, Z, nu, basis, level, rho_lo, rho_hi, log_rho_tol, sigma2, tree, tau)
        best[nu] = rho
        return val

    nu, val, _ = golden_max(profile, nu_lo, nu_hi, nu_tol)
    return nu, best[nu], val
