"""Quadratic form Q(rho) = Z_W^T C_W^-1 Z_W and dQ/dlog rho on the GPU:
against the dense oracle gradient, central differences (h = 1e-4) and the
autograd Functions."""
import math

import numpy as np
import pytest

from gpu_common import dev, host, require_gpu, say
from helpers import workload
from oracle import blup as OB

pytestmark = pytest.mark.gpu


def test_quad_form_and_gradient_vs_dense_oracle():
    torch = require_gpu()
    from paper_1701_00285_amd import PcgOptions, Solver
    wl = workload(4, n=4096, n_targets=1)       # the 4,096-point subsample
    say("grad cfg4 subsample")
    Q0, dQ0 = OB.quad_form_grad(wl.points, wl.z, wl.degree_w, wl.nu, wl.rho)
    s = Solver(wl.points, wl.degree_w, wl.leaf_max, wl.nu, wl.rho)
    zt = s.to_tree(dev(wl.z))
    opts = PcgOptions(rtol=1e-12, max_iter=5000)
    zw, _ = s.apply_W(zt)
    gw, info, _ = s.solve(zw, opts)
    gam = s.apply_Wt(gw)
    Q, dQ = s.quad_grad(zt, gam)
    assert Q == pytest.approx(Q0, rel=1e-8)
    assert dQ == pytest.approx(dQ0, rel=1e-8)
    # central differences of the GPU Q in log rho
    h = 1e-4
    qs = []
    for sgn in (1, -1):
        r = wl.rho * math.exp(sgn * h)
        gw2, _, _ = s.solve(zw, opts, rho=r)
        q2, _ = s.quad_grad(zt, s.apply_Wt(gw2), rho=r)
        qs.append(q2)
    assert (qs[0] - qs[1]) / (2 * h) == pytest.approx(dQ, rel=1e-5)


def test_autograd_functions():
    torch = require_gpu()
    from paper_1701_00285_amd import PcgOptions, Solver, autograd_functions
    BlupSolve, BlupQuadForm = autograd_functions()
    wl = workload(4, n=2000, n_targets=1)
    s = Solver(wl.points, wl.degree_w, wl.leaf_max, wl.nu, wl.rho)
    zt = s.to_tree(dev(wl.z))
    opts = PcgOptions(rtol=1e-12, max_iter=5000)
    lr = torch.tensor(math.log(wl.rho), dtype=torch.float64, device="cuda", requires_grad=True)
    Q = BlupQuadForm.apply(lr, zt, s, opts)
    Q.backward()
    g_quad = float(lr.grad)
    Q0, dQ0 = OB.quad_form_grad(wl.points, wl.z, wl.degree_w, wl.nu, wl.rho)
    assert float(Q.detach()) == pytest.approx(Q0, rel=1e-8)
    assert g_quad == pytest.approx(dQ0, rel=1e-8)
    # generic adjoint path: L = Z_W . gamma_W through BlupSolve (one extra solve)
    lr2 = torch.tensor(math.log(wl.rho), dtype=torch.float64, device="cuda", requires_grad=True)
    zw, _ = s.apply_W(zt)
    gw = BlupSolve.apply(lr2, zw, s, opts)
    (zw * gw).sum().backward()
    assert float(lr2.grad) == pytest.approx(dQ0, rel=1e-8)
