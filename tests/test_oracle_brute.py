"""Pins for oracle.brute: the fsum double loop, the row-block form and
scipy's cdist distances agree; special cases."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

import synth
from oracle import brute
from oracle.matern import matern, pairwise_dist


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
@pytest.mark.parametrize("deriv", [False, True])
def test_fsum_vs_blocks(nu, deriv):
    a = synth.uniform_cloud(37, 3, 11)
    b = synth.uniform_cloud(45, 3, 12)
    x = synth.standard_normal(45, 13)
    y1 = brute.fsum_matvec(a, b, x, nu, 0.2, 1.3, deriv=deriv)
    y2 = brute.cov_matvec(a, b, x, nu, 0.2, 1.3, deriv=deriv, block=8)
    np.testing.assert_allclose(y2, y1, rtol=1e-13, atol=1e-14)


def test_distances_vs_cdist():
    a = synth.uniform_cloud(50, 7, 1)
    b = synth.uniform_cloud(60, 7, 2)
    np.testing.assert_allclose(pairwise_dist(a, b), cdist(a, b), rtol=1e-14, atol=1e-15)


def test_self_pairs_and_empty():
    a = synth.uniform_cloud(20, 2, 4)
    x = np.ones(20)
    y = brute.cov_matvec(a, a, x, 0.5, 0.1)
    C = matern(cdist(a, a), 0.5, 0.1)
    np.testing.assert_allclose(y, C.sum(axis=1), rtol=1e-14)
    np.testing.assert_allclose(np.diag(C), 1.0, rtol=4e-16)
    assert brute.cov_matvec(a[:0], a, x, 0.5, 0.1).shape == (0,)
