"""Pins for oracle.likelihood: the restricted-likelihood determinant identity
and the GLS quadratic form at level 0, the white-noise closed form, the
nested condition numbers of the Proposition in Sec. 5.1, invariance under
rotations inside a cell, and the MLE being a local maximum.  For the
sparsified C~^n_W (Sec. 4.1): the tree search against a brute-force
region test over every node, points inside the widened box and the
descendants always found, a symmetric pattern that grows with tau and
covers everything for a tau larger than the domain, and the white-noise
closed form at tau = 0."""
import math

import numpy as np
import pytest

from helpers import workload
from oracle import blup as OB
from oracle import likelihood as OL
from oracle.basis import build_basis
from oracle.kdtree import build_kdtree
from oracle.matern import cov_matrix


def _case(k, n):
    wl = workload(k, n=n, n_targets=1)
    tree = build_kdtree(wl.points, wl.leaf_max)
    bas = build_basis(wl.points, tree, wl.degree_w)
    return wl, tree, bas


@pytest.mark.parametrize("k,n", [(1, 500), (2, 400)])
def test_level0_determinant_and_quadratic_form(k, n):
    wl, tree, bas = _case(k, n)
    l0, logdet, quad, nt = OL.multilevel_loglik(wl.points, wl.z, wl.nu, wl.rho, bas, 0)
    assert nt == n - bas.p
    ref = OL.reml_logdet(wl.points, wl.degree_w, wl.nu, wl.rho)
    assert abs(logdet - ref) < 1e-9 * abs(ref) + 1e-8
    q = OB.quad_form(wl.points, wl.z, wl.degree_w, wl.nu, wl.rho)
    assert abs(quad - q) < 1e-8 * abs(q)
    assert abs(l0 - (-0.5 * (nt * math.log(2 * math.pi) + ref + q))) < 1e-8 * abs(l0)


def test_white_noise_closed_form():
    # nu = 1/2 with rho far below the smallest distance: C = sigma2 I to rounding
    wl, tree, bas = _case(1, 300)
    dmin = min(np.min(np.linalg.norm(wl.points[i + 1:] - wl.points[i], axis=1)) for i in range(299))
    rho = dmin / 800.0
    sigma2 = 2.5
    C = cov_matrix(wl.points, wl.points, 0.5, rho, sigma2)
    assert np.max(np.abs(C - sigma2 * np.eye(300))) <= 4e-16 * sigma2
    for level in (tree.max_depth, 2, 0):
        l, logdet, quad, nt = OL.multilevel_loglik(wl.points, wl.z, 0.5, rho, bas, level, sigma2)
        zn = bas.W[:nt] @ wl.z
        assert abs(logdet - nt * math.log(sigma2)) < 1e-10 * nt
        assert abs(quad - float(zn @ zn) / sigma2) < 1e-11 * quad
        assert abs(l - (-0.5 * nt * (math.log(2 * math.pi) + math.log(sigma2)) - 0.5 * float(zn @ zn) / sigma2)) \
            < 1e-10 * abs(l)


def test_condition_numbers_nest():
    wl, tree, bas = _case(2, 500)
    C = cov_matrix(wl.points, wl.points, wl.nu, wl.rho)
    kap = []
    for level in range(tree.max_depth, -1, -1):
        nt = OL.level_rows(bas, level)
        ev = np.linalg.eigvalsh(bas.W[:nt] @ C @ bas.W[:nt].T)
        kap.append(ev[-1] / ev[0])
    ev = np.linalg.eigvalsh(C)
    kap.append(ev[-1] / ev[0])
    assert all(kap[i] <= kap[i + 1] * (1 + 1e-8) for i in range(len(kap) - 1)), kap


def test_rotation_inside_cells_leaves_loglik_unchanged():
    wl, tree, bas = _case(1, 400)
    rng = np.random.default_rng(5)
    W2 = bas.W.copy()
    for v, (off, cnt) in bas.node_rows.items():
        if cnt > 1:
            Q, _ = np.linalg.qr(rng.standard_normal((cnt, cnt)))
            W2[off:off + cnt] = Q @ W2[off:off + cnt]
    rot = OL.Basis(W=W2, L=bas.L, level_rows=bas.level_rows, node_rows=bas.node_rows, node_a=bas.node_a, p=bas.p)
    for level in (tree.max_depth, 1):
        a = OL.multilevel_loglik(wl.points, wl.z, wl.nu, wl.rho, bas, level)
        b = OL.multilevel_loglik(wl.points, wl.z, wl.nu, wl.rho, rot, level)
        assert abs(a[0] - b[0]) < 1e-9 * abs(a[0])


def test_mle_is_a_local_maximum():
    wl, tree, bas = _case(1, 300)
    level = tree.max_depth - 1
    rho, val, evals = OL.mle_rho(wl.points, wl.z, wl.nu, bas, level, 0.01, 1.0, 1e-5)
    assert 0.01 < rho < 1.0 and evals > 10
    for f in (math.exp(-1e-2), math.exp(1e-2)):
        assert OL.multilevel_loglik(wl.points, wl.z, wl.nu, rho * f, bas, level)[0] <= val


def test_golden_max_on_a_parabola():
    x, fx, evals = OL.golden_max(lambda t: -(t - 0.3) ** 2, -2.0, 5.0, 1e-8)
    assert abs(x - 0.3) < 1e-8 and fx <= 0.0 and evals > 30


def test_profile_mle_is_a_local_maximum_in_nu_and_rho():
    wl, tree, bas = _case(1, 200)
    level = tree.max_depth - 1
    nu, rho, val = OL.mle_nu_rho(wl.points, wl.z, bas, level, 0.3, 2.0, 0.02, 0.5, 2e-2, 2e-3)
    assert 0.3 < nu < 2.0 and 0.02 < rho < 0.5
    for dn, dr in ((0.05, 0.0), (-0.05, 0.0), (0.0, 0.03), (0.0, -0.03)):
        other = OL.multilevel_loglik(wl.points, wl.z, nu + dn, rho * math.exp(dr), bas, level)[0]
        assert other <= val + 1e-9 * abs(val)


# ---- sparsified C~^n_W (Sec. 4.1 tree search) ------------------------------------

def _parents(tree):
    par = [-1] * tree.n_nodes
    for v in range(tree.n_nodes):
        if not tree.is_leaf(v):
            par[tree.left[v]] = v
            par[tree.right[v]] = v
    return par


def _region(tree, par, b):
    """Per-axis (lower, upper) bounds of node b's region: the left side of a
    split is x_k <= s (closed), the right side x_k > s (open)."""
    lb = np.full(tree.d, -np.inf)
    ub = np.full(tree.d, np.inf)
    c = b
    while par[c] >= 0:
        u = par[c]
        k, s = tree.axis[u], tree.threshold[u]
        if tree.left[u] == c:
            ub[k] = min(ub[k], s)
        else:
            lb[k] = max(lb[k], s)
        c = u
    return lb, ub


@pytest.mark.parametrize("k,n", [(1, 500), (2, 400)])
def test_tree_search_is_the_widened_box_meeting_the_node_regions(k, n):
    wl, tree, bas = _case(k, n)
    par = _parents(tree)
    regions = [_region(tree, par, b) for b in range(tree.n_nodes)]
    for tau in (0.0, 0.03, 0.15):
        for a in range(tree.n_nodes):
            lo, hi = OL.node_box(wl.points, tree, a)
            for j in range(tree.depth[a], tree.max_depth + 1):
                got = sorted(OL.search_tree(tree, lo, hi, j, tau))
                want = [b for b in range(tree.n_nodes) if tree.depth[b] == j
                        and np.all(lo - tau <= regions[b][1]) and np.all(hi + tau > regions[b][0])]
                assert got == want, (tau, a, j)


def test_tree_search_finds_points_in_the_widened_box_and_the_descendants():
    wl, tree, bas = _case(2, 400)
    S = wl.points
    par = _parents(tree)
    for tau in (0.0, 0.05):
        for a in range(tree.n_nodes):
            lo, hi = OL.node_box(S, tree, a)
            for j in range(tree.depth[a], tree.max_depth + 1):
                got = set(OL.search_tree(tree, lo, hi, j, tau))
                for b in range(tree.n_nodes):
                    if tree.depth[b] != j:
                        continue
                    P = S[tree.perm[tree.begin[b]:tree.end[b]]]
                    inside = np.any(np.all((P >= lo - tau) & (P <= hi + tau), axis=1))
                    c = b
                    while c >= 0 and c != a:
                        c = par[c]
                    if inside or c == a:
                        assert b in got, (tau, a, j, b)


def test_sparsity_pattern_is_symmetric_monotone_and_full_for_large_tau():
    wl, tree, bas = _case(1, 500)
    level = 1
    nt = OL.level_rows(bas, level)
    prev = None
    for tau in (0.0, 0.02, 0.1, 0.3):
        m = OL.sparsity_mask(wl.points, tree, bas, level, tau)
        assert m.shape == (nt, nt) and np.array_equal(m, m.T)
        for v, (off, cnt) in bas.node_rows.items():
            if cnt and tree.depth[v] >= level:
                assert m[off:off + cnt, off:off + cnt].all()
        if prev is not None:
            assert np.all(m >= prev)
        prev = m
    assert prev.sum() < nt * nt
    # the unit square widened by 2 covers every region
    assert OL.sparsity_mask(wl.points, tree, bas, level, 2.0).all()
    a = OL.multilevel_loglik(wl.points, wl.z, wl.nu, wl.rho, bas, level, tree=tree, tau=2.0)
    b = OL.multilevel_loglik(wl.points, wl.z, wl.nu, wl.rho, bas, level)
    assert a == b


def test_sparsified_white_noise_closed_form():
    wl, tree, bas = _case(1, 300)
    dmin = min(np.min(np.linalg.norm(wl.points[i + 1:] - wl.points[i], axis=1)) for i in range(299))
    rho, sigma2 = dmin / 800.0, 2.5
    for level in (tree.max_depth, 0):
        l, logdet, quad, nt = OL.multilevel_loglik(wl.points, wl.z, 0.5, rho, bas, level, sigma2, tree, 0.0)
        zn = bas.W[:nt] @ wl.z
        assert abs(logdet - nt * math.log(sigma2)) < 1e-10 * nt
        assert abs(quad - float(zn @ zn) / sigma2) < 1e-11 * quad
