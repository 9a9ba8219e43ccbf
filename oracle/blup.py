"""Dense FP64 BLUP: classic formulae and the multilevel predictor.  TEST INFRASTRUCTURE.

Classic route (Sec. 2, eqs. GLSbeta and KrigBLUP):
    beta  = (X^T C^-1 X)^-1 X^T C^-1 Z
    gamma = C^-1 (Z - X beta)
    Zhat(x0) = k(x0)^T beta + c(x0)^T gamma
computed with the Cholesky factor G of C (A = G^-1 X, b = G^-1 Z, beta
from the least-squares problem min |A beta - b|, which has the same
normal equations as GLSbeta).

Multilevel route (Sec. 5.2, eqs. Spatial:problem and Spatial:eqn1-3): gamma
lies in the orthogonal complement of col(X), so gamma = W^T gamma_W with
    (W C W^T) gamma_W = W Z,
    beta = (X^T X)^-1 X^T (Z - C gamma)    (least squares on X),
which solves the saddle-point system exactly.  Here C_W is formed densely
from the explicit W of oracle.basis and factored by Cholesky.

Quadratic form and gradient (data term of the multilevel likelihood,
Sec. 3, l_W):  Q(rho) = Z_W^T C_W^-1 Z_W = Z^T gamma, and
    dQ / dlog rho = -gamma^T (rho dC/drho) gamma
(derivative of an inverse; W does not depend on rho).

Pins (tests/test_oracle_blup.py): saddle-point residual, classic ==
multilevel, exact interpolation at the data sites (no nugget),
reproduction of data drawn from the trend space, X^T gamma = 0, the
interpolation-residual identity |Zhat(S) - Z| = |W Z - C_W gamma_W|,
Q two ways, central differences of Q for the gradient.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .basis import Basis
from .design import design_matrix
from .matern import cov_matrix, cov_matrix_rho_drho


@dataclass
class BlupResult:
    beta: np.ndarray
    gamma: np.ndarray          # length N, input order
    zhat: np.ndarray | None    # predictions at targets
    gamma_w: np.ndarray | None = None


def classic_blup(S, Z, T, w, nu, rho, sigma2=1.0) -> BlupResult:
    S = np.asarray(S, dtype=np.float64)
    X = design_matrix(S, w)
    C = cov_matrix(S, S, nu, rho, sigma2)
    G = sla.cholesky(C, lower=True)
    A = sla.solve_triangular(G, X, lower=True)
    b = sla.solve_triangular(G, Z, lower=True)
    beta, *_ = np.linalg.lstsq(A, b, rcond=None)
    gamma = sla.cho_solve((G, True), Z - X @ beta)
    zhat = None
    if T is not None:
        zhat = design_matrix(T, w) @ beta + cov_matrix(T, S, nu, rho, sigma2) @ gamma
    return BlupResult(beta=beta, gamma=gamma, zhat=zhat)


def classic_blup_direct(S, Z, T, w, nu, rho, sigma2=1.0) -> BlupResult:
    """The classic formulae taken literally in FP64 (eqs. GLSbeta and
    KrigBLUP): C^-1 X and C^-1 Z by an LU solve with partial pivoting, then
    beta = (X^T C^-1 X)^-1 X^T C^-1 Z and gamma = C^-1 (Z - X beta).  This is
    the "traditional formulae in double precision" of the accuracy
    experiment (Sec. 8): unlike classic_blup it does not stop when C is not
    numerically positive definite."""
    S = np.asarray(S, dtype=np.float64)
    X = design_matrix(S, w)
    C = cov_matrix(S, S, nu, rho, sigma2)
    CiX = np.linalg.solve(C, X)
    CiZ = np.linalg.solve(C, Z)
    beta = np.linalg.solve(X.T @ CiX, X.T @ CiZ)
    gamma = np.linalg.solve(C, Z - X @ beta)
    zhat = None
    if T is not None:
        zhat = design_matrix(T, w) @ beta + cov_matrix(T, S, nu, rho, sigma2) @ gamma
    return BlupResult(beta=beta, gamma=gamma, zhat=zhat)


def multilevel_blup(S, Z, T, w, nu, rho, basis: Basis, sigma2=1.0) -> BlupResult:
    S = np.asarray(S, dtype=np.float64)
    X = design_matrix(S, w)
    C = cov_matrix(S, S, nu, rho, sigma2)
    W = basis.W
    CW = W @ C @ W.T
    ZW = W @ Z
    gw = sla.cho_solve(sla.cho_factor(CW, lower=True), ZW)
    gamma = W.T @ gw
    beta, *_ = np.linalg.lstsq(X, Z - C @ gamma, rcond=None)
    zhat = None
    if T is not None:
        zhat = design_matrix(T, w) @ beta + cov_matrix(T, S, nu, rho, sigma2) @ gamma
    return BlupResult(beta=beta, gamma=gamma, zhat=zhat, gamma_w=gw)


def quad_form(S, Z, w, nu, rho, sigma2=1.0) -> float:
    """Q = (Z - X beta)^T C^-1 (Z - X beta) with the GLS beta (classic route)."""
    res = classic_blup(S, Z, None, w, nu, rho, sigma2)
    return float(np.dot(Z, res.gamma))


def quad_form_grad(S, Z, w, nu, rho, sigma2=1.0) -> tuple[float, float]:
    """(Q, dQ/dlog rho) with dQ/dlog rho = -gamma^T (rho dC/drho) gamma."""
    res = classic_blup(S, Z, None, w, nu, rho, sigma2)
    Cd = cov_matrix_rho_drho(S, S, nu, rho, sigma2)
    return float(np.dot(Z, res.gamma)), float(-res.gamma @ (Cd @ res.gamma))
