"""Pins for oracle.likelihood: the restricted-likelihood determinant identity
and the GLS quadratic form at level 0, the white-noise closed form, the
nested condition numbers of the Proposition in Sec. 3, invariance under
rotations inside a cell, and the MLE being a local maximum."""
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
