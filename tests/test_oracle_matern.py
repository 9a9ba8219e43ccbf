"""Pins for oracle.matern: library routine (scipy K_nu through the
Definition), the nu = 1/2 special case, phi(0), derivative by differences,
and a planted mistake (the half-integer sum exactly as printed) that the
library pin must reject."""
import math

import numpy as np
import pytest

from oracle import matern as M

R = np.concatenate([[0.0, 1e-12, 1e-6, 1e-3], np.linspace(0.01, 3.0, 60), [5.0, 10.0, 30.0]])


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5, 3.5])
@pytest.mark.parametrize("rho", [0.1, 0.3, 1.0])
def test_halfint_matches_bessel_definition(nu, rho):
    a = M.matern(R, nu, rho)
    b = M.matern_bessel(R, nu, rho)
    np.testing.assert_allclose(a, b, rtol=5e-13, atol=1e-300)


def test_nu_half_is_exponential():
    for rho in (0.1, 0.5, 2.0):
        np.testing.assert_allclose(M.matern(R, 0.5, rho), np.exp(-R / rho), rtol=1e-15, atol=0)


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_value_at_zero_is_variance(nu):
    assert M.matern(np.array([0.0]), nu, 0.3, sigma2=2.5)[0] == pytest.approx(2.5, rel=1e-15)
    assert M.matern_rho_drho(np.array([0.0]), nu, 0.3, sigma2=2.5)[0] == 0.0


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_rho_derivative_central_difference(nu):
    rho, h = 0.3, 1e-5
    fd = (M.matern_bessel(R, nu, rho * math.exp(h)) - M.matern_bessel(R, nu, rho * math.exp(-h))) / (2 * h)
    np.testing.assert_allclose(M.matern_rho_drho(R, nu, rho), fd, rtol=1e-7, atol=1e-10)


def test_closed_forms_in_z():
    """Expanded forms in z = sqrt(2 nu) r / rho (the ones the device code uses)
    agree with the finite sum and with K_nu."""
    z = np.linspace(0, 8, 41)
    for nu, val, der in [
        (0.5, np.exp(-z), z * np.exp(-z)),
        (1.5, (1 + z) * np.exp(-z), z * z * np.exp(-z)),
        (2.5, (1 + z + z * z / 3) * np.exp(-z), z * z * (1 + z) / 3 * np.exp(-z)),
    ]:
        rho = 0.7
        r = z * rho / math.sqrt(2 * nu)
        np.testing.assert_allclose(M.matern(r, nu, rho), val, rtol=1e-14, atol=1e-300)
        np.testing.assert_allclose(M.matern_bessel(r, nu, rho), val, rtol=1e-13, atol=1e-300)
        np.testing.assert_allclose(M.matern_rho_drho(r, nu, rho), der, rtol=1e-13, atol=1e-300)


def test_planted_mistake_printed_sum_is_rejected(monkeypatch):
    """The half-integer sum as printed (k from 1, (n+1)! in the numerator)
    must fail the K_nu pin; this shows the pin can see such a mistake."""
    def printed_coefs(n):
        return [0.0] + [math.factorial(n + 1) / (math.factorial(k) * math.factorial(n - k)) * 2.0 ** (-k)
                        for k in range(1, n + 1)]
    monkeypatch.setattr(M, "_coefs", printed_coefs)
    a = M.matern(R[1:], 1.5, 0.3)
    b = M.matern_bessel(R[1:], 1.5, 0.3)
    assert not np.allclose(a, b, rtol=1e-3)


def test_gaussian_is_the_large_nu_limit_of_the_definition():
    """nu = +inf (Gaussian, Sec. 8 accuracy experiment) against the kv form
    of the Definition at large nu: the gap shrinks like 1/nu."""
    r = np.linspace(0.0, 3.0, 31)
    g = M.matern(r, np.inf, 0.7, 1.3)
    assert g[0] == 1.3
    gaps = []
    for nu in (25.0, 50.0, 100.0):          # the kv form overflows Gamma(nu) beyond nu ~ 170
        b = M.matern_bessel(r, nu, 0.7, 1.3)
        gaps.append(np.max(np.abs(b - g)))
    assert gaps[2] < 4e-3
    for a, b in zip(gaps, gaps[1:]):        # O(1/nu): the gap halves when nu doubles
        assert 1.8 < a / b < 2.2
    np.testing.assert_allclose(g, 1.3 * np.exp(-r ** 2 / (2 * 0.49)), rtol=4e-15)


def test_gaussian_rho_derivative_central_difference():
    r = np.linspace(0.01, 2.5, 40)
    rho, h = 0.6, 1e-6
    fd = rho * (M.matern(r, np.inf, rho * (1 + h)) - M.matern(r, np.inf, rho * (1 - h))) / (2 * rho * h)
    np.testing.assert_allclose(M.matern_rho_drho(r, np.inf, rho), fd, rtol=1e-7, atol=1e-10)


@pytest.mark.parametrize("nu", [0.3, 0.75, 1.0, 1.25, 2.2, 4.0])
def test_general_nu_rho_derivative_central_difference(nu):
    """rho d phi / d rho from the Bessel-derivative identity against central
    differences of the Definition in log rho (any nu, including integer nu
    where K_{nu-1} has integer order and nu < 1 where the order is negative)."""
    from oracle.matern import matern_bessel, matern_bessel_rho_drho, matern_rho_drho
    r = np.linspace(0.0, 2.0, 41)
    rho, h = 0.4, 1e-5
    fd = (matern_bessel(r, nu, rho * np.exp(h)) - matern_bessel(r, nu, rho * np.exp(-h))) / (2 * h)
    d = matern_bessel_rho_drho(r, nu, rho)
    assert np.max(np.abs(d - fd)) < 1e-8
    assert d[0] == 0.0
    assert np.array_equal(matern_rho_drho(r, nu, rho), d)
