"""Brute-force covariance sums y_i = sum_j phi(|x_i - y_j|) a_j.  TEST INFRASTRUCTURE.

The dense product C(theta) x is the dominant step of every iteration of
the predictor's Krylov solve (Sec. 6.2, three-step product W^T -> C -> W).
Two plain forms:

  fsum_matvec  pure-Python double loop, distances by math.sqrt of summed
               squared differences, row sums by math.fsum (correctly
               rounded) -- for n <= ~64;
  cov_matvec   NumPy row blocks of the dense covariance block times x,
               FP64 throughout, distances from differences.  This is the
               CPU baseline the benchmark times.

Pins (tests/test_oracle_brute.py): the two forms agree; scipy.spatial's
cdist distances; symmetric / self-pair / empty special cases.
"""
from __future__ import annotations

import math

import numpy as np

from .matern import matern, matern_rho_drho


def fsum_matvec(rows, cols, x, nu, rho, sigma2=1.0, deriv=False):
    f = matern_rho_drho if deriv else matern
    out = []
    for xi in rows:
        terms = []
        for xj, aj in zip(cols, x):
            r = math.sqrt(sum((float(u) - float(v)) ** 2 for u, v in zip(xi, xj)))
            terms.append(float(f(np.array([r]), nu, rho, sigma2)[0]) * float(aj))
        out.append(math.fsum(terms))
    return np.array(out, dtype=np.float64)


def cov_matvec(rows, cols, x, nu, rho, sigma2=1.0, deriv=False, block=256):
    rows = np.asarray(rows, dtype=np.float64)
    cols = np.asarray(cols, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    f = matern_rho_drho if deriv else matern
    y = np.empty(rows.shape[0])
    for s in range(0, rows.shape[0], block):
        blk = rows[s:s + block]
        r2 = np.zeros((blk.shape[0], cols.shape[0]))
        for k in range(cols.shape[1]):
            diff = blk[:, k][:, None] - cols[:, k][None, :]
            r2 += diff * diff
        y[s:s + block] = f(np.sqrt(r2), nu, rho, sigma2) @ x
    return y
