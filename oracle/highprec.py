"""Classic BLUP in high-precision arithmetic (mpmath).  TEST INFRASTRUCTURE.

The reference of the accuracy experiment (Sec. 8, "Prediction numerical
accuracy under ill-conditioning"): the paper compares the double-precision
results with a 52-digit solution of the classic formulae (Sec. 2, eqs.
GLSbeta and KrigBLUP),
    beta  = (X^T C^-1 X)^-1 X^T C^-1 Z,   gamma = C^-1 (Z - X beta),
    Zhat(x0) = k(x0)^T beta + c(x0)^T gamma,
for the Gaussian kernel phi(r) = exp(-r^2 / (2 theta^2)).  Here every
step runs in mpmath at `dps` significant digits from the FP64 inputs taken
exactly: C and c(x0) entry by entry, X with the graded-lex monomials of
oracle.design (same order), C^-1 [X | Z] through the Cholesky factor of C
(C is positive definite in exact arithmetic; the Gaussian matrices of the
experiment have condition numbers far beyond 1e19, the largest FP64 can
show, and need about 100 digits), and the p x p system by an LU solve.

Pins (tests/test_oracle_highprec.py): agreement with the FP64 oracle on a
well-conditioned case, and the interpolation property Zhat(S) = Z.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np

from .design import td_exponents


def _mono(x, exps):
    out = []
    for e in exps:
        v = mp.mpf(1)
        for xi, ei in zip(x, e):
            if ei:
                v *= xi ** ei
        out.append(v)
    return out


def gaussian_blup(S, Z, T, w: int, theta: float, dps: int = 60):
    """(beta, zhat, beta_str, zhat_str, kappa_lb): beta over the graded-lex
    monomials and zhat at the targets T, as FP64 arrays rounded from the
    `dps`-digit results and as 25-digit strings; kappa_lb = (max g_ii /
    min g_ii)^2 over the Cholesky factor, a lower bound on cond_2(C)."""
    with mp.workdps(dps):
        S = [[mp.mpf(float(v)) for v in row] for row in np.asarray(S, dtype=np.float64)]
        T = [[mp.mpf(float(v)) for v in row] for row in np.asarray(T, dtype=np.float64)]
        Z = [mp.mpf(float(v)) for v in np.asarray(Z, dtype=np.float64)]
        n, d = len(S), len(S[0])
        exps = td_exponents(d, w)
        p = len(exps)
        h = 1 / (2 * mp.mpf(float(theta)) ** 2)

        def kern(a, b):
            return mp.exp(-h * sum((ai - bi) ** 2 for ai, bi in zip(a, b)))

        # Cholesky C = G G^T, in place (lower triangle)
        G = [[mp.mpf(0)] * n for _ in range(n)]
        for i in range(n):
            for j in range(i + 1):
                s = kern(S[i], S[j]) - mp.fsum(G[i][k] * G[j][k] for k in range(j))
                if i == j:
                    if s <= 0:
                        raise ArithmeticError("covariance matrix not positive definite at this precision")
                    G[i][i] = mp.sqrt(s)
                else:
                    G[i][j] = s / G[j][j]

        def csolve(b):
            y = [mp.mpf(0)] * n
            for i in range(n):
                y[i] = (b[i] - mp.fsum(G[i][k] * y[k] for k in range(i))) / G[i][i]
            x = [mp.mpf(0)] * n
            for i in range(n - 1, -1, -1):
                x[i] = (y[i] - mp.fsum(G[k][i] * x[k] for k in range(i + 1, n))) / G[i][i]
            return x

        X = [_mono(s, exps) for s in S]
        CiX = [csolve([X[i][j] for i in range(n)]) for j in range(p)]   # columns
        CiZ = csolve(Z)
        M = mp.matrix(p, p)
        r = mp.matrix(p, 1)
        for a in range(p):
            for b in range(p):
                M[a, b] = mp.fsum(X[i][a] * CiX[b][i] for i in range(n))
            r[a] = mp.fsum(X[i][a] * CiZ[i] for i in range(n))
        beta = mp.lu_solve(M, r)
        res = [Z[i] - mp.fsum(X[i][a] * beta[a] for a in range(p)) for i in range(n)]
        gamma = csolve(res)
        zhat = []
        for t in T:
            kt = _mono(t, exps)
            zhat.append(mp.fsum(kt[a] * beta[a] for a in range(p)) + mp.fsum(kern(t, S[i]) * gamma[i]
                                                                            for i in range(n)))
        diag = [G[i][i] for i in range(n)]
        kappa_lb = (max(diag) / min(diag)) ** 2
        return (np.array([float(beta[a]) for a in range(p)]), np.array([float(v) for v in zhat]),
                [mp.nstr(beta[a], 25) for a in range(p)], [mp.nstr(v, 25) for v in zhat], mp.nstr(kappa_lb, 6))


def gaussian_cov_in_basis(S, P, theta: float, T=None, dps: int = 40):
    """P C P^T (and K(T, S) P^T when targets T are given) for the Gaussian
    kernel exp(-r^2 / (2 theta^2)), every entry formed at `dps` digits from
    the FP64 sites and the FP64 rows of P taken exactly, then rounded to FP64.
    With P = [W; L] the multilevel basis (Sec. 3.1) this is C_W and its
    companions of Sec. 5.2, free of the rounding that FP64 products leave
    when W's vanishing moments cancel the kernel's low-degree part (the
    accuracy experiment of Sec. 8)."""
    with mp.workdps(dps):
        S = [[mp.mpf(float(v)) for v in row] for row in np.asarray(S, dtype=np.float64)]
        P = [[mp.mpf(float(v)) for v in row] for row in np.asarray(P, dtype=np.float64)]
        h = 1 / (2 * mp.mpf(float(theta)) ** 2)

        def kern(a, b):
            return mp.exp(-h * mp.fsum((ai - bi) ** 2 for ai, bi in zip(a, b)))

        n = len(S)
        C = [[kern(S[i], S[j]) for j in range(n)] for i in range(n)]
        CPt = [[mp.fdot(C[i], P[r]) for r in range(len(P))] for i in range(n)]
        G = np.array([[float(mp.fdot(P[r], [CPt[i][s] for i in range(n)])) for s in range(len(P))]
                      for r in range(len(P))])
        if T is None:
            return G
        T = [[mp.mpf(float(v)) for v in row] for row in np.asarray(T, dtype=np.float64)]
        KPt = np.array([[float(mp.fdot([kern(t, S[j]) for j in range(n)], P[r])) for r in range(len(P))] for t in T])
        return G, KPt
