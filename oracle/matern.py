"""Matern covariance for half-integer smoothness, FP64.  TEST INFRASTRUCTURE.

Paper: Definition (Sec. 3.1, "Binary multilevel basis") gives
    phi(r) = (sqrt(2 nu) r / rho)^nu K_nu(sqrt(2 nu) r / rho) / (Gamma(nu) 2^(nu-1)),
and the remark after it states that for nu = n + 1/2 the function is an
exponential times a finite sum.  The printed sum is garbled (index starts
at 1, "(n+1)!" where "(n+k)!" belongs); this module uses the standard
finite expansion of the half-integer Bessel function (Abramowitz & Stegun
10.2.15 / 10.1.9):
    K_{n+1/2}(z) = sqrt(pi / (2 z)) e^{-z} sum_{k=0}^{n} (n+k)! / (k! (n-k)!) (2 z)^{-k}.
Substituting into the Definition with z = sqrt(2 nu) r / rho gives
    phi(r) = sigma2 * c_n * e^{-z} * sum_{k=0}^{n} (n+k)!/(k!(n-k)!) 2^{-k} z^{n-k},
    c_n = sqrt(pi/2) / (Gamma(n + 1/2) 2^{n - 1/2}).
A variance sigma2 multiplies the Definition (phi(0) = sigma2); the paper's
Definition is the sigma2 = 1 case.

Derivative used by the gradient: rho d phi / d rho = -u m'(u) with u = r/rho
and m the sigma2 = 1 shape; with P(z) the finite sum above,
    rho d phi/d rho = sigma2 * c_n * z e^{-z} (P(z) - P'(z)).

nu = +inf: the Definition's limit as nu grows without bound, in this
parametrisation, is the Gaussian kernel
    phi(r) = sigma2 exp(-r^2 / (2 rho^2)),   rho d phi/d rho = (r/rho)^2 phi,
the kernel of the accuracy experiment in Sec. 8 (there with theta = rho).

Pins (tests/test_oracle_matern.py): scipy.special.kv through the
Definition; nu = 1/2 reduces to exp(-r/rho); phi(0) = sigma2; derivative
against central differences of the kv form; the Gaussian against the kv
form at large nu.
"""
from __future__ import annotations

import math

import numpy as np


def _halfint_n(nu: float) -> int:
    n = nu - 0.5
    if n < 0 or abs(n - round(n)) > 1e-12:
        raise ValueError(f"nu={nu} is not a half-integer >= 1/2")
    return int(round(n))


def _coefs(n: int):
    """Coefficients of P(z) = sum_k a_k z^{n-k}, a_k = (n+k)!/(k!(n-k)!) 2^{-k}."""
    return [math.factorial(n + k) / (math.factorial(k) * math.factorial(n - k)) * 2.0 ** (-k)
            for k in range(n + 1)]


def _prefactor(n: int) -> float:
    return math.sqrt(math.pi / 2.0) / (math.gamma(n + 0.5) * 2.0 ** (n - 0.5))


def matern(r, nu: float, rho: float, sigma2: float = 1.0):
    """phi(r) for nu = n + 1/2 (Definition + half-integer remark, Sec. 3.1),
    the Gaussian limit for nu = +inf, and the Definition itself (scipy's
    K_nu, `matern_bessel`) for any other nu > 0."""
    if math.isinf(nu) and nu > 0:
        r = np.asarray(r, dtype=np.float64)
        return sigma2 * np.exp(-(r / rho) ** 2 / 2.0)
    if abs(nu - 0.5 - round(nu - 0.5)) > 1e-12:
        return matern_bessel(r, nu, rho, sigma2)
    n = _halfint_n(nu)
    r = np.asarray(r, dtype=np.float64)
    z = math.sqrt(2.0 * nu) * r / rho
    P = np.zeros_like(z)
    for k, a in enumerate(_coefs(n)):
        P = P + a * z ** (n - k)
    return sigma2 * _prefactor(n) * np.exp(-z) * P


def matern_rho_drho(r, nu: float, rho: float, sigma2: float = 1.0):
    """rho * d phi / d rho at fixed r (used for the log-rho gradient)."""
    if math.isinf(nu) and nu > 0:
        r = np.asarray(r, dtype=np.float64)
        u2 = (r / rho) ** 2
        return sigma2 * u2 * np.exp(-u2 / 2.0)
    if abs(nu - 0.5 - round(nu - 0.5)) > 1e-12:
        return matern_bessel_rho_drho(r, nu, rho, sigma2)
    n = _halfint_n(nu)
    r = np.asarray(r, dtype=np.float64)
    z = math.sqrt(2.0 * nu) * r / rho
    P = np.zeros_like(z)
    dP = np.zeros_like(z)
    for k, a in enumerate(_coefs(n)):
        e = n - k
        P = P + a * z ** e
        if e > 0:
            dP = dP + a * e * z ** (e - 1)
    return sigma2 * _prefactor(n) * z * np.exp(-z) * (P - dP)


def matern_bessel(r, nu: float, rho: float, sigma2: float = 1.0):
    """The Definition evaluated with scipy's K_nu (any nu > 0); r = 0 -> sigma2.
    Used only as an independent pin for `matern`."""
    from scipy.special import gamma, kv
    r = np.asarray(r, dtype=np.float64)
    z = np.sqrt(2.0 * nu) * r / rho
    out = np.full_like(z, sigma2)
    nz = z > 0
    out[nz] = sigma2 * (z[nz] ** nu) * kv(nu, z[nz]) / (gamma(nu) * 2.0 ** (nu - 1.0))
    return out


def matern_bessel_rho_drho(r, nu: float, rho: float, sigma2: float = 1.0):
    """rho d phi / d rho for any nu > 0 from the Definition: with
    z = sqrt(2 nu) r / rho, rho d/d rho = -z d/dz, and the derivative of the
    Bessel product, d/dz [z^nu K_nu(z)] = -z^nu K_{nu-1}(z) (Abramowitz &
    Stegun 9.6.28 with K_{-mu} = K_mu), gives
        rho d phi / d rho = sigma2 z^(nu+1) K_{nu-1}(z) / (Gamma(nu) 2^(nu-1)),
    zero at r = 0.  scipy's K_nu as in `matern_bessel`."""
    from scipy.special import gamma, kv
    r = np.asarray(r, dtype=np.float64)
    z = np.sqrt(2.0 * nu) * r / rho
    out = np.zeros_like(z)
    nz = z > 0
    out[nz] = sigma2 * (z[nz] ** (nu + 1.0)) * kv(nu - 1.0, z[nz]) / (gamma(nu) * 2.0 ** (nu - 1.0))
    return out


def pairwise_dist(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Euclidean distances from coordinate differences (never the Gram form)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    r2 = np.zeros((a.shape[0], b.shape[0]))
    for k in range(a.shape[1]):
        diff = a[:, k][:, None] - b[:, k][None, :]
        r2 += diff * diff
    return np.sqrt(r2)


def cov_matrix(a, b, nu, rho, sigma2=1.0):
    """Dense block {phi(|a_i - b_j|)} (Sec. 3.1, item ii of the notation)."""
    return matern(pairwise_dist(a, b), nu, rho, sigma2)


def cov_matrix_rho_drho(a, b, nu, rho, sigma2=1.0):
    """Dense block {rho d phi/d rho (|a_i - b_j|)}."""
    return matern_rho_drho(pairwise_dist(a, b), nu, rho, sigma2)
