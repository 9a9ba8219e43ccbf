"""Device W / W^T transform against the invariants and the oracle's
projection onto the trend space."""
import math

import numpy as np
import pytest

import synth
from gpu_common import dev, host, require_gpu, say
from oracle.design import design_matrix

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,d,w,leaf", [(1000, 2, 1, 32), (3000, 3, 2, 64), (2051, 5, 1, 20), (777, 10, 1, 64),
                                        (65536, 3, 2, 64)])
def test_transform_invariants(n, d, w, leaf):
    torch = require_gpu()
    from paper_1701_00285_amd import Solver
    say(f"transform n={n} d={d} w={w} leaf={leaf}")
    pts = synth.uniform_cloud(n, d, n + d)
    s = Solver(pts, w, leaf, 1.5, 0.2)
    Xt = design_matrix(pts[s.tree.perm], w)                 # tree order
    scale = np.abs(Xt).max() * math.sqrt(n)
    for k in range(Xt.shape[1]):                             # vanishing moments
        vw, _ = s.apply_W(dev(Xt[:, k]))
        assert np.abs(host(vw)).max() < 1e-11 * scale
    v = synth.standard_normal(n, 4)
    vw, vl = s.apply_W(dev(v))
    # isometry and the oracle's projection onto col(X): |W v|^2 = |v|^2 - |P_X v|^2
    proj = Xt @ np.linalg.lstsq(Xt, v, rcond=None)[0]
    assert float(np.sum(host(vl) ** 2)) == pytest.approx(float(proj @ proj), rel=1e-10)
    assert float(np.sum(host(vw) ** 2)) == pytest.approx(float(v @ v - proj @ proj), rel=1e-10)
    back = s.apply_Wt(vw, vl)                                 # W^T W v + L^T L v = v
    np.testing.assert_allclose(host(back), v, atol=1e-12 * np.abs(v).max())
    back_w = host(s.apply_Wt(vw))                             # W^T W v = v - P_X v
    np.testing.assert_allclose(back_w, v - proj, atol=1e-10 * np.abs(v).max())
    if n <= 3000:                                              # against the dense host basis
        W, Lm = s.basis.dense()
        np.testing.assert_allclose(host(vw), W @ v, atol=1e-12 * np.abs(v).max() * math.sqrt(n))
        u = synth.standard_normal(n - s.p, 5)
        np.testing.assert_allclose(host(s.apply_Wt(dev(u))), W.T @ u, atol=1e-12 * math.sqrt(n))
