"""Test-side helpers that combine the seeded generators with the oracle."""
import numpy as np
import scipy.linalg as sla

import synth
from oracle.design import design_matrix
from oracle.matern import cov_matrix


def workload(k, n=None, n_targets=None):
    """Workload k with Z filled in.  For workload 1 the correlated part of Z
    is G xi with G = chol(C), C from the oracle's covariance function."""
    wl = synth.make_config(k, n=n, n_targets=n_targets)
    if wl.z is None:
        X = design_matrix(wl.points, wl.degree_w)
        C = cov_matrix(wl.points, wl.points, wl.nu, wl.rho, wl.sigma2)
        G = sla.cholesky(C, lower=True)
        beta = wl.extra["beta_gen"][: X.shape[1]]
        wl.z = X @ beta + G @ wl.extra["xi"]
    return wl


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)
