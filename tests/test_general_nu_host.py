"""General smoothness nu (not a half-integer, Definition of Sec. 3.1): the
library's table evaluation (the code the FP64 pair kernels run, here on the
host) against the Definition through scipy's K_nu."""
import numpy as np
import pytest

from oracle.matern import matern_bessel


@pytest.mark.parametrize("nu", [0.3, 0.75, 1.0, 1.25, 2.0, 3.0, 3.5, 3.7, 6.2, 8.0])
def test_table_matches_the_definition(nu):
    from paper_1701_00285_amd import matern_host
    z = np.concatenate([np.linspace(0.0, 2.0, 2001), np.linspace(2.0, 70.0, 8001)])
    r = z * 0.8 / np.sqrt(2 * nu)
    a = matern_host(r, nu, 0.8, 1.7)
    b = matern_bessel(r, nu, 0.8, 1.7)
    assert a[0] == pytest.approx(1.7, rel=1e-15)
    live = b > 1.7e-17
    assert np.max(np.abs(a[live] - b[live]) / b[live]) < 1.5e-13
    # entries below 1e-18 sigma2 are dropped (set to zero), nothing else is
    assert np.all(a[~live] <= 1.7e-17) and np.all(a[b > 1.7e-18] > 0)


def test_near_integer_nu_loses_digits_as_stated():
    from paper_1701_00285_amd import matern_host
    z = np.linspace(0.0, 6.0, 3001)
    r = z / np.sqrt(2 * 0.999)
    assert np.max(np.abs(matern_host(r, 0.999, 1.0) - matern_bessel(r, 0.999, 1.0))) < 5e-12


def test_half_integer_and_gaussian_closed_forms_on_the_host():
    from paper_1701_00285_amd import matern_host
    from oracle.matern import matern
    r = np.linspace(0, 4, 81)
    for nu in (0.5, 1.5, 2.5, np.inf):
        np.testing.assert_allclose(matern_host(r, nu, 0.6, 1.1), matern(r, nu, 0.6, 1.1), rtol=2e-15, atol=1e-300)


def test_out_of_range_nu_is_rejected():
    from paper_1701_00285_amd import MlblupError, matern_host
    for nu in (0.0, -1.0, 8.5, 20.0):
        with pytest.raises(MlblupError, match="EINVAL"):
            matern_host(np.ones(3), nu, 1.0)
