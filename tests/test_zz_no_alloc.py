"""The covariance product on the library's static scratch
(mlblup_cov_matvec_noalloc) against the product with a caller workspace
(mlblup_cov_matvec): two calls in a row on each path, the second on a smaller
input, so that what the first call left in the shared scratch is there when
the second runs.  The two entry points share their kernels and schedule, so
the outputs must agree bit for bit; the FP64 values are also held against the
oracle's row-block sums on sampled rows (same bar as the product tests).  A
product larger than the static scratch is refused."""
import numpy as np
import pytest

import synth
from gpu_common import dev, host, require_gpu, row_relerr, say
from oracle import brute
from oracle.matern import matern, pairwise_dist

pytestmark = pytest.mark.gpu


def _pair(rows, cols, x, nu, rho, s2, prec, outputs):
    from paper_1701_00285_amd import cov_matvec, cov_matvec_noalloc
    y_ref, dy_ref = cov_matvec(rows, cols, x, nu, rho, s2, precision=prec, outputs=outputs)
    y, dy = cov_matvec_noalloc(rows, cols, x, nu, rho, s2, precision=prec, outputs=outputs)
    return (y_ref, dy_ref), (y, dy)


def _same(a, b):
    return a is None and b is None or bool((a == b).all())


CASES = [
    # (m, n, d, nu, rho, precision, outputs, square): the first of each pair is
    # the larger; the second runs right after it on the same scratch
    ((20000, 20000, 3, 1.5, 0.2, 0, 1, True), (17000, 17000, 3, 1.5, 0.2, 0, 1, True)),
    ((18000, 18000, 10, 0.5, 0.5, 3, 1, True), (3000, 5000, 10, 0.5, 0.5, 3, 1, False)),
    ((4000, 9000, 5, 2.5, 0.3, 0, 3, False), (1000, 1500, 5, 2.5, 0.3, 1, 3, False)),
]


@pytest.mark.parametrize("pair", CASES, ids=["sym_fp64_then_smaller", "mfma_sym_then_rect", "rect_both_outputs"])
def test_noalloc_matches_workspace_entry(pair):
    torch = require_gpu()
    from paper_1701_00285_amd import FP64
    for k, (m, n, d, nu, rho, prec, outputs, square) in enumerate(pair):
        say(f"noalloc call {k}: m={m} n={n} d={d} nu={nu} precision={prec} outputs={outputs}")
        cols_h = synth.uniform_cloud(n, d, 100 + d + k)
        rows_h = cols_h if square else synth.uniform_cloud(m, d, 200 + d + k)
        x_h = synth.standard_normal(n, 300 + k)
        cols = dev(cols_h)
        rows = cols if square else dev(rows_h)
        x = dev(x_h)
        (y0, dy0), (y1, dy1) = _pair(rows, cols, x, nu, rho, 1.3, prec, outputs)
        torch.cuda.synchronize()
        assert _same(y0, y1) and _same(dy0, dy1), f"call {k}: outputs differ from the workspace entry point"
        if prec == FP64 and outputs & 1:
            idx = np.random.default_rng(k).choice(m, 12, replace=False)
            ref = brute.cov_matvec(rows_h[idx], cols_h, x_h, nu, rho, 1.3)
            sc = 1.3 * np.abs(matern(pairwise_dist(rows_h[idx], cols_h), nu, rho)) @ np.abs(x_h)
            err = row_relerr(host(y1)[idx], ref, sc)
            say(f"  sampled rows vs oracle: {err:.2e}")
            assert err < 1e-13


def test_noalloc_refuses_products_above_the_scratch():
    torch = require_gpu()
    from paper_1701_00285_amd import FP64, MlblupError, cov_matvec_noalloc, cov_workspace_bytes
    from paper_1701_00285_amd.api import NOALLOC_SCRATCH_BYTES
    n, d = 240000, 3
    assert cov_workspace_bytes(n, n, d, FP64) > NOALLOC_SCRATCH_BYTES
    pts = torch.zeros((n, d), dtype=torch.float64, device="cuda")
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(MlblupError, match="static"):
        cov_matvec_noalloc(pts, pts, x, 1.5, 0.2)
    # the entry point still works after the refusal
    small = dev(synth.uniform_cloud(64, d, 5))
    xs = dev(synth.standard_normal(64, 6))
    y, _ = cov_matvec_noalloc(small, small, xs, 1.5, 0.2)
    torch.cuda.synchronize()
    ref = brute.fsum_matvec(host(small), host(small), host(xs), 1.5, 0.2)
    assert np.max(np.abs(host(y) - ref)) < 1e-13 * np.max(np.abs(ref)) * 64
