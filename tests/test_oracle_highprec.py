"""The high-precision classic BLUP (reference of the accuracy experiment,
Sec. 8) and what FP64 does on that experiment."""
import numpy as np
import pytest

import synth
from conftest import ROOT
from oracle import blup as B
from oracle import highprec as H
from oracle.basis import build_basis
from oracle.kdtree import build_kdtree
from oracle.matern import cov_matrix


def _reference():
    ref, lines = {}, open(f"{ROOT}/tests/golden/gaussian_accuracy_reference.txt").read().split("\n")
    i = 0
    while i < len(lines):
        if lines[i].startswith("case"):
            a, th = map(float, lines[i].split()[1:])
            ref[(a, th)] = dict(checksum=float(lines[i + 1].split()[1]), kappa_lower=float(lines[i + 2].split()[1]),
                                beta=np.array([float(v) for v in lines[i + 3].split()[1:]]),
                                zhat=np.array([float(v) for v in lines[i + 4].split()[1:]]))
            i += 5
        else:
            i += 1
    return ref


def _rel(x, y):
    return np.linalg.norm(x - y) / np.linalg.norm(y)


def test_highprec_matches_fp64_oracle_when_well_conditioned():
    g = np.random.default_rng(3)
    S, T = synth.unit_disk(60, g), synth.unit_disk(20, g)
    Z = 1 + np.sin(S[:, 0]) * np.sin(S[:, 1])
    b, z, *_ = H.gaussian_blup(S, Z, T, 2, 0.3, dps=40)
    ref = B.classic_blup(S, Z, T, 2, np.inf, 0.3)          # cond(C) ~ 1e8
    assert _rel(b, ref.beta) < 1e-10 and _rel(z, ref.zhat) < 1e-10


def test_highprec_interpolates_the_data():
    g = np.random.default_rng(4)
    S = synth.unit_disk(50, g)
    Z = 1 + np.sin(2 * S[:, 0]) * np.sin(2 * S[:, 1])
    _, z, *_ = H.gaussian_blup(S, Z, S, 3, 1.0, dps=60)      # targets = sites: Zhat(S) = Z (no nugget)
    np.testing.assert_allclose(z, Z, rtol=0, atol=1e-15)


def test_golden_reference_inputs_and_one_case_recomputed():
    ref = _reference()
    assert list(ref) == [tuple(c) for c in synth.ACCURACY_CASES]
    for (a, th), r in ref.items():
        pts, tgt, _ = synth.accuracy_experiment(a)
        assert float(np.sum(pts) + np.sum(tgt)) == r["checksum"]
    a, th = 0.5, 3.0
    pts, tgt, z = synth.accuracy_experiment(a)
    b, zh, *_ = H.gaussian_blup(pts, z, tgt, 8, th, dps=100)
    assert _rel(b, ref[(a, th)]["beta"]) < 1e-15 and _rel(zh, ref[(a, th)]["zhat"]) < 1e-15


def test_fp64_behaviour_on_the_accuracy_experiment():
    """What double precision does here: cond(C) is far beyond 1e19 (the
    Cholesky diagonal alone bounds it by >= 1e49), C_W = W C W^T formed in
    FP64 is rounding noise (indefinite), and the classic formulae solved by
    LU with pivoting still give the predictions to the accuracy below."""
    ref = _reference()
    bound = {(1.0, 10.0): 1e-6, (0.5, 10.0): 1e-8, (2.0, 10.0): 1e-3, (2.0, 3.0): 1e-3, (0.5, 3.0): 1e-8}
    for (a, th), r in ref.items():
        assert r["kappa_lower"] > 1e49
        pts, tgt, z = synth.accuracy_experiment(a)
        c = B.classic_blup_direct(pts, z, tgt, 8, np.inf, th)
        assert _rel(c.zhat, r["zhat"]) < bound[(a, th)]
    pts, _, _ = synth.accuracy_experiment(1.0)
    W = build_basis(pts, build_kdtree(pts, 64), 8).W
    ev = np.linalg.eigvalsh(W @ cov_matrix(pts, pts, np.inf, 10.0) @ W.T)
    assert ev[0] < 0 < ev[-1] and ev[-1] < 1e-13


def test_cov_in_basis_matches_fp64_when_no_cancellation():
    """A rough Gaussian (theta = 0.05) and a random orthogonal P: nothing
    cancels, so the high-precision P C P^T equals the FP64 product to FP64
    rounding; the trace is that of C (N, since phi(0) = 1) for orthogonal P."""
    g = np.random.default_rng(11)
    S, T = synth.unit_disk(30, g), synth.unit_disk(5, g)
    P, _ = np.linalg.qr(g.standard_normal((30, 30)))
    G, KP = H.gaussian_cov_in_basis(S, P, 0.05, T=T, dps=40)
    C = cov_matrix(S, S, np.inf, 0.05)
    ref = P @ C @ P.T
    assert np.max(np.abs(G - ref)) < 1e-14 * np.max(np.abs(C))
    assert np.max(np.abs(KP - cov_matrix(T, S, np.inf, 0.05) @ P.T)) < 1e-14
    assert abs(np.trace(G) - 30.0) < 1e-12
    assert np.max(np.abs(G - G.T)) < 1e-15


def test_cov_in_basis_shows_the_cancellation_of_flat_kernels():
    """With the multilevel basis of degree w = 4 and a flat Gaussian
    (theta = 3), W C W^T is the part of the kernel above degree 4: the
    high-precision block is about 1e-8 of C and positive definite (smallest
    eigenvalue ~1e-23), while the FP64 product carries rounding of about
    1e-16 of C on top of it, which makes it indefinite."""
    g = np.random.default_rng(12)
    S = synth.unit_disk(60, g)
    tree = build_kdtree(S, 16)
    basis = build_basis(S, tree, 4)
    W, Lm = basis.W, basis.L
    P = np.vstack([W, Lm])                  # columns in input order
    G = H.gaussian_cov_in_basis(S, P, 3.0, dps=40)
    m = W.shape[0]
    Cw = G[:m, :m]
    assert np.linalg.eigvalsh(Cw)[0] > 0
    fp = (W @ cov_matrix(S, S, np.inf, 3.0) @ W.T)
    assert np.max(np.abs(Cw)) < 1e-6
    assert 1e-18 < np.max(np.abs(fp - Cw)) < 1e-13
    assert np.linalg.eigvalsh(fp)[0] < 0
