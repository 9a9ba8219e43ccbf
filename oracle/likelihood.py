"""Multilevel log-likelihood and its maximum in rho.  TEST INFRASTRUCTURE.

Paper, Sec. 3 (the reduced multilevel likelihoods that follow the
multilevel likelihood): for a level n, the partial transform
W^n = [W_t; ...; W_n] (the first N~ rows of W, finest level first) gives

    l_n(theta) = -N~/2 log(2 pi) - 1/2 log det C^n_W - 1/2 (Z^n_W)^T (C^n_W)^-1 Z^n_W,

with C^n_W = W^n C (W^n)^T and Z^n_W = W^n Z.  Sec. 7 (estimator
computation) takes the determinant and the quadratic form from one
Cholesky factor G of C^n_W: log det = 2 sum log G_ii and the quadratic form
is |G^-1 Z^n_W|^2.  Here C^n_W is formed densely from the oracle's explicit
W (per-cell SVD, oracle.basis); the paper's sparsification of C_W is not
applied, so this is the exact value.

The maximum over rho (nu, sigma2 fixed) is found by golden-section search
on log rho, the textbook method (Kiefer 1953): keep the two interior points
of a bracket at the golden ratio and drop the side whose interior point is
lower.

Pins (tests/test_oracle_likelihood.py): at n = 0 the determinant obeys the
restricted-likelihood identity log det(W C W^T) = log det C
+ log det(X^T C^-1 X) - log det(X^T X) (P = [W; L] orthogonal, L spanning the
columns of X), and the quadratic form equals the GLS residual form of
oracle.blup; with C = sigma2 I the value has a closed form; the condition
numbers nest as the Proposition of Sec. 3 states; rotations of the wavelets
inside a cell leave l_n unchanged; the MLE is a local maximum.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .basis import Basis
from .design import design_matrix
from .matern import cov_matrix

LOG_2PI = math.log(2.0 * math.pi)


def level_rows(basis: Basis, level: int) -> int:
    """N~: number of wavelet rows at levels >= level."""
    return int(sum(r for q, r in basis.level_rows.items() if q >= level))


def multilevel_loglik(S, Z, nu, rho, basis: Basis, level: int, sigma2=1.0):
    """(l_n, log det C^n_W, (Z^n_W)^T (C^n_W)^-1 Z^n_W, N~) for the points S
    (input order, the order of basis.W's columns) and data Z."""
    S = np.asarray(S, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    nt = level_rows(basis, level)
    Wn = basis.W[:nt]
    C = cov_matrix(S, S, nu, rho, sigma2)
    Cn = Wn @ C @ Wn.T
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
            sigma2=1.0):
    """rho maximising l_level (golden section on log rho): (rho, l, evaluations)."""
    def f(lr):
        return multilevel_loglik(S, Z, nu, math.exp(lr), basis, level, sigma2)[0]

    lr, val, evals = golden_max(f, math.log(rho_lo), math.log(rho_hi), log_tol)
    return math.exp(lr), val, evals


def mle_nu_rho(S, Z, basis: Basis, level: int, nu_lo: float, nu_hi: float, rho_lo: float, rho_hi: float,
               nu_tol: float = 1e-3, log_rho_tol: float = 1e-4, sigma2=1.0):
    """(nu, rho) maximising l_level by the profile likelihood: golden
    section over nu, each point the golden-section rho maximum.  Returns
    (nu, rho, l)."""
    best = {}

    def profile(nu):
        rho, val, _ = mle_rho(S, Z, nu, basis, level, rho_lo, rho_hi, log_rho_tol, sigma2)
        best[nu] = rho
        return val

    nu, val, _ = golden_max(profile, nu_lo, nu_hi, nu_tol)
    return nu, best[nu], val
