"""Pins for oracle.blup: saddle-point system, classic == multilevel, exact
interpolation (no nugget), trend reproduction, X^T gamma = 0, the
interpolation-residual identity, Q two ways, gradient by differences."""
import math

import numpy as np
import pytest

import synth
from helpers import relerr, workload
from oracle import blup as OB
from oracle.basis import build_basis
from oracle.design import design_matrix
from oracle.kdtree import build_kdtree
from oracle.matern import cov_matrix


def _small(k, n, nt=50):
    wl = workload(k, n=n, n_targets=nt)
    tree = build_kdtree(wl.points, wl.leaf_max)
    bas = build_basis(wl.points, tree, wl.degree_w)
    return wl, tree, bas


@pytest.mark.parametrize("k,n", [(1, 1000), (2, 700), (4, 500)])
def test_saddle_point_and_routes_agree(k, n):
    wl, tree, bas = _small(k, n)
    S, Z = wl.points, wl.z
    cl = OB.classic_blup(S, Z, wl.targets, wl.degree_w, wl.nu, wl.rho)
    ml = OB.multilevel_blup(S, Z, wl.targets, wl.degree_w, wl.nu, wl.rho, bas)
    X = design_matrix(S, wl.degree_w)
    C = cov_matrix(S, S, wl.nu, wl.rho)
    # saddle point system [C X; X^T 0][gamma; beta] = [Z; 0]
    assert relerr(C @ cl.gamma + X @ cl.beta, Z) < 1e-10
    assert np.abs(X.T @ cl.gamma).max() < 1e-8 * np.abs(cl.gamma).max() * n
    assert relerr(C @ ml.gamma + X @ ml.beta, Z) < 1e-10
    assert np.abs(X.T @ ml.gamma).max() < 1e-9 * np.abs(ml.gamma).max() * n
    assert relerr(ml.beta, cl.beta) < 1e-8
    assert relerr(ml.gamma, cl.gamma) < 1e-8
    assert relerr(ml.zhat, cl.zhat) < 1e-9


def test_exact_interpolation_at_data_sites():
    wl, tree, bas = _small(1, 1000)
    ml = OB.multilevel_blup(wl.points, wl.z, wl.points, wl.degree_w, wl.nu, wl.rho, bas)
    assert relerr(ml.zhat, wl.z) < 1e-11


def test_trend_reproduction():
    wl, tree, bas = _small(2, 600)
    X = design_matrix(wl.points, wl.degree_w)
    beta0 = synth.standard_normal(X.shape[1], 7)
    Z = X @ beta0
    ml = OB.multilevel_blup(wl.points, Z, wl.targets, wl.degree_w, wl.nu, wl.rho, bas)
    assert relerr(ml.beta, beta0) < 1e-11
    assert np.abs(ml.gamma).max() < 1e-9
    np.testing.assert_allclose(ml.zhat, design_matrix(wl.targets, wl.degree_w) @ beta0, rtol=1e-10, atol=1e-10)


def test_interpolation_residual_identity():
    """With an inexact gamma_W: |Zhat(S) - Z| = |W Z - C_W gamma_W|."""
    wl, tree, bas = _small(2, 400)
    S, Z = wl.points, wl.z
    X = design_matrix(S, wl.degree_w)
    C = cov_matrix(S, S, wl.nu, wl.rho)
    W = bas.W
    gw = np.linalg.solve(W @ C @ W.T, W @ Z) + 1e-3 * synth.standard_normal(W.shape[0], 1)
    gamma = W.T @ gw
    beta, *_ = np.linalg.lstsq(X, Z - C @ gamma, rcond=None)
    zs = X @ beta + C @ gamma
    lhs = np.linalg.norm(zs - Z)
    rhs = np.linalg.norm(W @ Z - W @ C @ W.T @ gw)
    assert lhs == pytest.approx(rhs, rel=1e-9)


def test_quad_form_two_ways_and_gradient():
    wl, tree, bas = _small(4, 400)
    S, Z = wl.points, wl.z
    Q, dQ = OB.quad_form_grad(S, Z, wl.degree_w, wl.nu, wl.rho)
    ml = OB.multilevel_blup(S, Z, None, wl.degree_w, wl.nu, wl.rho, bas)
    assert float(np.dot(bas.W @ Z, ml.gamma_w)) == pytest.approx(Q, rel=1e-9)
    h = 1e-4
    qp = OB.quad_form(S, Z, wl.degree_w, wl.nu, wl.rho * math.exp(h))
    qm = OB.quad_form(S, Z, wl.degree_w, wl.nu, wl.rho * math.exp(-h))
    assert (qp - qm) / (2 * h) == pytest.approx(dQ, rel=1e-6)
