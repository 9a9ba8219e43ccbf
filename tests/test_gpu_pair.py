"""Pair kernel (dense Matern product) on the GPU against the oracle:
brute-force fsum sums for n <= 64, row-block FP64 sums at several tiles
with ragged tails, sampled rows at the full 65,536-point size, special
cases and determinism."""
import numpy as np
import pytest

import synth
from gpu_common import dev, host, require_gpu, row_relerr, say
from oracle import brute
from oracle.matern import matern, pairwise_dist

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-13      # relative to sum_j |phi_ij x_j|
FP32_TOL = 2e-6


def _scale(rows, cols, x, nu, rho):
    return np.abs(matern(pairwise_dist(rows, cols), nu, rho)) @ np.abs(x)


@pytest.mark.parametrize("d", [1, 2, 3, 5, 7, 10, 20])
@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5, np.inf])
def test_brute_force_small(d, nu):
    torch = require_gpu()
    from paper_1701_00285_amd import DLOGRHO, FP32, FP64, VALUE, cov_matvec
    m, n = 41, 64
    rows = synth.uniform_cloud(m, d, 10 + d)
    cols = synth.uniform_cloud(n, d, 20 + d)
    x = synth.standard_normal(n, 30 + d)
    rho, s2 = 0.3 * np.sqrt(d), 1.7
    say(f"pair brute d={d} nu={nu}")
    ref = brute.fsum_matvec(rows, cols, x, nu, rho, s2)
    dref = brute.fsum_matvec(rows, cols, x, nu, rho, s2, deriv=True)
    sc = s2 * _scale(rows, cols, x, nu, rho)
    for prec, tol in ((FP64, FP64_TOL), (FP32, FP32_TOL)):
        y, dy = cov_matvec(dev(rows), dev(cols), dev(x), nu, rho, s2, precision=prec, outputs=VALUE | DLOGRHO)
        torch.cuda.synchronize()
        assert row_relerr(host(y), ref, sc) < tol
        assert row_relerr(host(dy), dref, sc) < tol
        y1, _ = cov_matvec(dev(rows), dev(cols), dev(x), nu, rho, s2, precision=prec, outputs=VALUE)
        _, dy2 = cov_matvec(dev(rows), dev(cols), dev(x), nu, rho, s2, precision=prec, outputs=DLOGRHO)
        assert np.array_equal(host(y1), host(y)) and np.array_equal(host(dy2), host(dy))


@pytest.mark.parametrize("m,n,d", [(3000, 2500, 3), (1537, 4099, 2), (2049, 1031, 5), (700, 900, 10), (513, 700, 20)])
def test_several_tiles_ragged(m, n, d):
    torch = require_gpu()
    from paper_1701_00285_amd import FP32, FP64, cov_matvec
    rows = synth.uniform_cloud(m, d, 1)
    cols = synth.uniform_cloud(n, d, 2)
    x = synth.standard_normal(n, 3)
    for nu in (0.5, 1.5, 2.5, np.inf):
        rho = 0.2 * np.sqrt(d)
        say(f"pair tiles m={m} n={n} d={d} nu={nu}")
        ref = brute.cov_matvec(rows, cols, x, nu, rho)
        sc = _scale(rows, cols, x, nu, rho)
        y, _ = cov_matvec(dev(rows), dev(cols), dev(x), nu, rho, precision=FP64)
        assert row_relerr(host(y), ref, sc) < FP64_TOL
        y, _ = cov_matvec(dev(rows), dev(cols), dev(x), nu, rho, precision=FP32)
        assert row_relerr(host(y), ref, sc) < FP32_TOL


def test_self_product_exact_diagonal_and_determinism():
    torch = require_gpu()
    from paper_1701_00285_amd import FP32, FP64, cov_matvec
    pts = synth.uniform_cloud(1000, 3, 5)
    x = np.zeros(1000)
    x[17] = 1.0
    for prec in (FP64, FP32):
        y, _ = cov_matvec(dev(pts), dev(pts), dev(x), 0.5, 0.1, 2.0, precision=prec)
        col = host(y)
        assert col[17] == 2.0                      # sigma2 * phi(0), exactly
    x = synth.standard_normal(1000, 6)
    a, _ = cov_matvec(dev(pts), dev(pts), dev(x), 1.5, 0.2)
    b, _ = cov_matvec(dev(pts), dev(pts), dev(x), 1.5, 0.2)
    assert np.array_equal(host(a), host(b))


def test_empty_inputs():
    torch = require_gpu()
    from paper_1701_00285_amd import cov_matvec
    pts = dev(synth.uniform_cloud(10, 2, 1))
    y, _ = cov_matvec(pts, pts[:0], dev(np.zeros(0)), 0.5, 0.1)
    assert np.all(host(y) == 0.0)
    y, _ = cov_matvec(pts[:0], pts, dev(np.ones(10)), 0.5, 0.1)
    assert y.numel() == 0


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_full_size_sampled_rows(k):
    """Every workload at full size, in the launches the solve and the bench
    use: the square product on the tree-ordered points in every precision
    that applies to the workload, and the FP64 target product, checked on
    sampled rows computed one by one by the oracle."""
    torch = require_gpu()
    from paper_1701_00285_amd import FP32, FP64, MFMA_BF16X3, MFMA_FP32, Tree, cov_matvec
    wl = synth.make_config(k, with_z=False)
    pts = wl.points[Tree(wl.points, wl.leaf_max).perm]
    x = synth.standard_normal(wl.n, 77)
    nrow = 32 if wl.n <= 600_000 else 12   # the oracle's rows stay within seconds
    idx = np.random.default_rng(k).choice(wl.n, nrow, replace=False)
    say(f"pair full size cfg{k} n={wl.n} d={wl.d}")
    ref = brute.cov_matvec(pts[idx], pts, x, wl.nu, wl.rho)
    sc = _scale(pts[idx], pts, x, wl.nu, wl.rho)
    P, X = dev(pts), dev(x)
    precs = [(FP64, FP64_TOL), (FP32, FP32_TOL)]
    if 8 <= wl.d <= 32:
        precs += [(MFMA_FP32, 2e-5), (MFMA_BF16X3, 3e-4)]
    for prec, tol in precs:
        y, _ = cov_matvec(P, P, X, wl.nu, wl.rho, precision=prec)
        err = row_relerr(host(y)[idx], ref, sc)
        say(f"  precision={prec}: max row error {err:.2e}")
        assert err < tol, prec
    it = np.random.default_rng(k + 10).choice(wl.targets.shape[0], nrow // 2, replace=False)
    tref = brute.cov_matvec(wl.targets[it], pts, x, wl.nu, wl.rho)
    tsc = _scale(wl.targets[it], pts, x, wl.nu, wl.rho)
    yt, _ = cov_matvec(dev(wl.targets), P, X, wl.nu, wl.rho, precision=FP64)
    assert row_relerr(host(yt)[it], tref, tsc) < FP64_TOL


@pytest.mark.parametrize("n,d", [(16384, 3), (16385, 5), (16897, 3), (17408, 5), (16385, 10), (16896, 20),
                                 (16385, 7), (16896, 25)])
def test_symmetric_square_product(n, d):
    """Square products (rows and cols the same array, n >= 16,384) take the
    symmetric path; ragged last block, odd and even numbers of blocks; d = 7
    and 25 run in the kernels compiled for 8 and 28 with zero-padded
    coordinates.  The oracle checks 96 sampled rows (full rows of the
    product)."""
    torch = require_gpu()
    from paper_1701_00285_amd import DLOGRHO, FP32, FP64, VALUE, cov_matvec
    pts = synth.uniform_cloud(n, d, 40 + n)
    x = synth.standard_normal(n, 41 + n)
    say(f"symmetric n={n} d={d}")
    idx = np.unique(np.concatenate([np.arange(0, n, max(1, n // 64)), np.arange(n - 32, n)]))
    for nu in (0.5, 1.5, 2.5, np.inf):
        rho = 0.25 * np.sqrt(d / 3)
        ref = brute.cov_matvec(pts[idx], pts, x, nu, rho, 1.3)
        dref = brute.cov_matvec(pts[idx], pts, x, nu, rho, 1.3, deriv=True)
        sc = 1.3 * _scale(pts[idx], pts, x, nu, rho)
        P, X = dev(pts), dev(x)
        for prec, tol in ((FP64, FP64_TOL), (FP32, FP32_TOL)):
            y, dy = cov_matvec(P, P, X, nu, rho, 1.3, precision=prec, outputs=VALUE | DLOGRHO)
            assert row_relerr(host(y)[idx], ref, sc) < tol
            assert row_relerr(host(dy)[idx], dref, sc) < tol
            y1, _ = cov_matvec(P, P, X, nu, rho, 1.3, precision=prec, outputs=VALUE)
            assert np.array_equal(host(y1), host(y))
            # the row-tiled path on a copy of the same points agrees everywhere
            yr, _ = cov_matvec(P, P.clone(), X, nu, rho, 1.3, precision=prec)
            full_scale, _ = cov_matvec(P, P.clone(), torch.abs(X), nu, rho, 1.3, precision=FP64)
            assert row_relerr(host(yr), host(y1), host(full_scale)) < 2 * tol


@pytest.mark.parametrize("d", [8, 12, 20, 25])
def test_symmetric_expanded_distance_near_pairs(d):
    """From d = 8 on the FP64 square product forms squared distances as
    |a|^2 + |b|^2 - 2 a.b relative to each row block's first point and
    recomputes the pairs where that form cancels.  Points in tight clusters
    (spreads 1e-7 .. 1e-2) around centres far apart, shuffled so that most
    near pairs sit far from their block's first point, plus exact duplicates:
    the cancelling pairs are many and must still match the oracle to the
    FP64 tolerance, duplicates giving phi(0) exactly."""
    torch = require_gpu()
    from paper_1701_00285_amd import DLOGRHO, FP64, VALUE, cov_matvec
    g = np.random.default_rng(300 + d)
    n, nc = 16896, 48
    centres = 4.0 * g.random((nc, d))
    lab = g.integers(0, nc, n)
    spread = np.array([1e-7, 1e-5, 1e-3, 1e-2])[lab % 4]
    pts = centres[lab] + spread[:, None] * g.standard_normal((n, d))
    dup = g.choice(n, 800, replace=False)
    pts[dup[:400]] = pts[dup[400:]]
    x = synth.standard_normal(n, 301 + d)
    say(f"expanded distance near pairs n={n} d={d}")
    idx = np.unique(np.concatenate([np.arange(0, n, n // 48), dup[:40], dup[400:440]]))
    P, X = dev(pts), dev(x)
    for nu in (0.5, 2.5, np.inf):
        rho = 0.02 if nu == np.inf else 0.05
        ref = brute.cov_matvec(pts[idx], pts, x, nu, rho, 1.0)
        dref = brute.cov_matvec(pts[idx], pts, x, nu, rho, 1.0, deriv=True)
        sc = _scale(pts[idx], pts, x, nu, rho)
        y, dy = cov_matvec(P, P, X, nu, rho, 1.0, precision=FP64, outputs=VALUE | DLOGRHO)
        assert row_relerr(host(y)[idx], ref, sc) < FP64_TOL, nu
        assert row_relerr(host(dy)[idx], dref, sc) < FP64_TOL, nu
        # against the row-tiled path (differences throughout) on every row
        yr, _ = cov_matvec(P, P.clone(), X, nu, rho, 1.0, precision=FP64)
        full_scale, _ = cov_matvec(P, P.clone(), torch.abs(X), nu, rho, 1.0, precision=FP64)
        assert row_relerr(host(y), host(yr), host(full_scale)) < 2 * FP64_TOL, nu


@pytest.mark.parametrize("d", [8, 10, 16, 20, 25])
@pytest.mark.parametrize("square", [False, True])
def test_matrix_core_gram(d, square):
    """Distance Gram on the matrix cores (FP32 and BF16 x3), rectangular and
    square (the square case takes exact differences on the near tiles),
    against the oracle; the self pair stays exact."""
    torch = require_gpu()
    from paper_1701_00285_amd import MFMA_BF16X3, MFMA_FP32, cov_matvec
    n = 3001
    cols = synth.uniform_cloud(n, d, 60 + d)
    rows = cols if square else synth.uniform_cloud(777, d, 61 + d)
    x = synth.standard_normal(n, 62 + d)
    idx = np.arange(0, rows.shape[0], 7)
    say(f"mfma d={d} square={square}")
    for nu in (0.5, 1.5, 2.5):
        rho = 0.35 * np.sqrt(d)
        ref = brute.cov_matvec(rows[idx], cols, x, nu, rho)
        sc = _scale(rows[idx], cols, x, nu, rho)
        R = dev(rows)
        C = R if square else dev(cols)
        for prec, tol in ((MFMA_FP32, 2e-5), (MFMA_BF16X3, 3e-4)):
            y, _ = cov_matvec(R, C, dev(x), nu, rho, precision=prec)
            assert row_relerr(host(y)[idx], ref, sc) < tol, (prec, nu)
    if square:
        e = np.zeros(n)
        e[1234] = 1.0
        for prec in (MFMA_FP32, MFMA_BF16X3):
            y, _ = cov_matvec(R, R, dev(e), 0.5, 1.0, 1.0, precision=prec)
            assert host(y)[1234] == 1.0


@pytest.mark.parametrize("n,d", [(16385, 10), (17000, 20), (16384, 8)])
def test_matrix_core_symmetric(n, d):
    """Square products in the matrix-core precisions at n >= 16,384 take the
    symmetric matrix-core kernel (tournament schedule, exact diagonal
    tiles); sampled rows against the oracle, self pair exact."""
    torch = require_gpu()
    from paper_1701_00285_amd import MFMA_BF16X3, MFMA_FP32, cov_matvec
    pts = synth.uniform_cloud(n, d, 70 + d)
    x = synth.standard_normal(n, 71 + d)
    idx = np.unique(np.concatenate([np.arange(0, n, max(1, n // 48)), np.arange(n - 16, n)]))
    say(f"mfma symmetric n={n} d={d}")
    P, X = dev(pts), dev(x)
    for nu in (0.5, 2.5):
        rho = 0.35 * np.sqrt(d)
        ref = brute.cov_matvec(pts[idx], pts, x, nu, rho)
        sc = _scale(pts[idx], pts, x, nu, rho)
        for prec, tol in ((MFMA_FP32, 2e-5), (MFMA_BF16X3, 3e-4)):
            y, _ = cov_matvec(P, P, X, nu, rho, precision=prec)
            err = row_relerr(host(y)[idx], ref, sc)
            say(f"  nu={nu} precision={prec}: max row error {err:.2e}")
            assert err < tol, (prec, nu)
            y2, _ = cov_matvec(P, P, X, nu, rho, precision=prec)
            assert np.array_equal(host(y), host(y2))
    e = np.zeros(n)
    e[n // 3] = 1.0
    for prec in (MFMA_FP32, MFMA_BF16X3):
        y, _ = cov_matvec(P, P, dev(e), 0.5, 1.0, 1.0, precision=prec)
        assert host(y)[n // 3] == 1.0


def test_gaussian_in_matrix_core_precisions_uses_the_fp32_kernels():
    """The matrix cores take the half-integer forms only; a Gaussian product
    asked in a matrix-core precision runs the FP32 kernels (FP32 tolerance)."""
    torch = require_gpu()
    from paper_1701_00285_amd import MFMA_BF16X3, MFMA_FP32, cov_matvec
    for n in (3001, 16385):
        pts = synth.uniform_cloud(n, 10, 90 + n)
        x = synth.standard_normal(n, 91)
        idx = np.arange(0, n, max(1, n // 40))
        rho = 0.4 * np.sqrt(10)
        ref = brute.cov_matvec(pts[idx], pts, x, np.inf, rho)
        sc = _scale(pts[idx], pts, x, np.inf, rho)
        P = dev(pts)
        for prec in (MFMA_FP32, MFMA_BF16X3):
            y, _ = cov_matvec(P, P, dev(x), np.inf, rho, precision=prec)
            assert row_relerr(host(y)[idx], ref, sc) < FP32_TOL


GENERAL_TOL = 2e-13   # per-entry table error <= 1.5e-13 relative (host test), then FP64 sums


@pytest.mark.parametrize("nu", [0.75, 1.0, 1.25, 3.5])
def test_general_nu_products(nu):
    """A smoothness outside the closed forms (Definition of Sec. 3.1, the
    paper's experiments use 0.75, 1 and 1.25): FP64 products from the table
    on the row-tiled path (brute force and several tiles) and the symmetric
    path, against the Definition through scipy's K_nu."""
    torch = require_gpu()
    from paper_1701_00285_amd import FP64, cov_matvec
    for (m, n, d) in ((41, 64, 2), (700, 1031, 3), (513, 700, 10)):
        rows = synth.uniform_cloud(m, d, 100 + d)
        cols = synth.uniform_cloud(n, d, 101 + d)
        x = synth.standard_normal(n, 102 + d)
        rho = 0.3 * np.sqrt(d)
        say(f"general nu={nu} m={m} n={n} d={d}")
        ref = brute.cov_matvec(rows, cols, x, nu, rho, 1.4)
        sc = 1.4 * _scale(rows, cols, x, nu, rho)
        y, _ = cov_matvec(dev(rows), dev(cols), dev(x), nu, rho, 1.4, precision=FP64)
        assert row_relerr(host(y), ref, sc) < GENERAL_TOL
    n = 16385
    pts = synth.uniform_cloud(n, 3, 103)
    x = synth.standard_normal(n, 104)
    idx = np.unique(np.concatenate([np.arange(0, n, n // 40), np.arange(n - 8, n)]))
    ref = brute.cov_matvec(pts[idx], pts, x, nu, 0.25)
    sc = _scale(pts[idx], pts, x, nu, 0.25)
    P = dev(pts)
    y, _ = cov_matvec(P, P, dev(x), nu, 0.25, precision=FP64)
    assert row_relerr(host(y)[idx], ref, sc) < GENERAL_TOL
    yr, _ = cov_matvec(P, P.clone(), dev(x), nu, 0.25, precision=FP64)       # row-tiled on a copy
    assert row_relerr(host(yr), host(y), host(cov_matvec(P, P.clone(), torch.abs(dev(x)), nu, 0.25)[0])) < GENERAL_TOL


GENERAL_FP32_TOL = 2e-5   # FP32 series / tables: ~1e-6 per value, a few 1e-6 from s^nu at tiny s


@pytest.mark.parametrize("nu", [0.75, 1.0, 1.25, 3.5])
def test_general_nu_fp32_and_derivative_products(nu):
    """General smoothness beyond FP64 values: the FP32 kernel values (series
    at the origin with hardware log2 / exp2, FP32 tables beyond; the
    matrix-core precisions take the same FP32 path) and the rho-derivative
    rho dphi/drho = sigma2 z^{nu+1} K_{nu-1}(z) (FP64 and FP32), against the
    oracle's Definition through scipy's K_nu and K_{nu-1}, on the row-tiled
    path and a square product at 16,385 points."""
    torch = require_gpu()
    from paper_1701_00285_amd import DLOGRHO, FP32, FP64, MFMA_BF16X3, VALUE, cov_matvec
    for (m, n, d) in ((41, 64, 2), (700, 1031, 3), (513, 700, 10)):
        rows = synth.uniform_cloud(m, d, 200 + d)
        cols = synth.uniform_cloud(n, d, 201 + d)
        x = synth.standard_normal(n, 202 + d)
        rho = 0.3 * np.sqrt(d)
        say(f"general nu={nu} fp32 / derivative m={m} n={n} d={d}")
        ref = brute.cov_matvec(rows, cols, x, nu, rho, 1.4)
        dref = brute.cov_matvec(rows, cols, x, nu, rho, 1.4, deriv=True)
        sc = 1.4 * _scale(rows, cols, x, nu, rho)
        y64, dy64 = cov_matvec(dev(rows), dev(cols), dev(x), nu, rho, 1.4, precision=FP64, outputs=VALUE | DLOGRHO)
        assert row_relerr(host(y64), ref, sc) < GENERAL_TOL
        assert row_relerr(host(dy64), dref, sc) < GENERAL_TOL
        for prec in (FP32, MFMA_BF16X3):
            y, dy = cov_matvec(dev(rows), dev(cols), dev(x), nu, rho, 1.4, precision=prec, outputs=VALUE | DLOGRHO)
            assert row_relerr(host(y), ref, sc) < GENERAL_FP32_TOL
            assert row_relerr(host(dy), dref, sc) < GENERAL_FP32_TOL
    n = 16385
    pts = synth.uniform_cloud(n, 3, 203)
    x = synth.standard_normal(n, 204)
    idx = np.unique(np.concatenate([np.arange(0, n, n // 40), np.arange(n - 8, n)]))
    ref = brute.cov_matvec(pts[idx], pts, x, nu, 0.25)
    dref = brute.cov_matvec(pts[idx], pts, x, nu, 0.25, deriv=True)
    sc = _scale(pts[idx], pts, x, nu, 0.25)
    P = dev(pts)
    y, dy = cov_matvec(P, P, dev(x), nu, 0.25, precision=FP32, outputs=VALUE | DLOGRHO)
    assert row_relerr(host(y)[idx], ref, sc) < GENERAL_FP32_TOL
    assert row_relerr(host(dy)[idx], dref, sc) < GENERAL_FP32_TOL
    _, dy64 = cov_matvec(P, P, dev(x), nu, 0.25, precision=FP64, outputs=DLOGRHO)
    assert row_relerr(host(dy64)[idx], dref, sc) < GENERAL_TOL