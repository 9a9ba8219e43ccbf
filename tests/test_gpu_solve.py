"""Solve, predict and the error paths on the GPU against the oracle's
dense classic BLUP and its invariants."""
import numpy as np
import pytest

import synth
from gpu_common import dev, host, require_gpu, say
from helpers import relerr, workload
from oracle import blup as OB
from oracle.design import design_matrix

pytestmark = pytest.mark.gpu


def _solver(wl, max_targets=0, leaf=None, nu=None):
    from paper_1701_00285_amd import Solver
    return Solver(wl.points, wl.degree_w, leaf or wl.leaf_max, wl.nu if nu is None else nu, wl.rho, wl.sigma2,
                  max_targets=max_targets)


@pytest.mark.parametrize("k,n,nt", [(1, None, None), (2, 3000, 500), (4, 2500, 300), (3, 2000, 200), (5, 1500, 100)])
def test_predict_matches_classic_oracle_fp64(k, n, nt):
    torch = require_gpu()
    from paper_1701_00285_amd import FP64, PcgOptions
    wl = workload(k, n=n, n_targets=nt)
    say(f"predict fp64 cfg{k} n={wl.n}")
    ref = OB.classic_blup(wl.points, wl.z, wl.targets, wl.degree_w, wl.nu, wl.rho)
    s = _solver(wl, max_targets=wl.targets.shape[0])
    out = s.predict(dev(wl.z), dev(wl.targets), PcgOptions(rtol=1e-13, max_iter=5000, precision=FP64))
    assert out["info"]["relres_fp64"] <= 1e-13
    assert relerr(host(out["zhat"]), ref.zhat) < 1e-10
    assert relerr(out["beta"], ref.beta) < 1e-9
    assert relerr(host(out["gamma"]), ref.gamma) < 1e-9
    # interpolation-residual identity |Zhat(S) - Z| = |r_W| and X^T gamma = 0
    X = design_matrix(wl.points, wl.degree_w)
    g = host(out["gamma"])
    assert np.abs(X.T @ g).max() < 1e-9 * np.abs(X).max() * np.abs(g).sum()


def test_predict_relres_1e8_and_interpolation_identity():
    torch = require_gpu()
    from paper_1701_00285_amd import PcgOptions
    wl = workload(1)
    s = _solver(wl, max_targets=wl.n)
    out = s.predict(dev(wl.z), dev(wl.points), PcgOptions(rtol=1e-8))
    info = out["info"]
    assert info["relres_fp64"] <= 1e-8
    zs = host(out["zhat"])
    assert np.linalg.norm(zs - wl.z) == pytest.approx(out["interp_res"], rel=1e-6, abs=1e-12)
    assert out["interp_res"] <= 1e-8 * info["zw_norm"] * 1.0000001


def test_trend_reproduction():
    torch = require_gpu()
    from paper_1701_00285_amd import PcgOptions
    wl = workload(2, n=2000, n_targets=100)
    X = design_matrix(wl.points, wl.degree_w)
    beta0 = synth.standard_normal(X.shape[1], 8)
    z = X @ beta0
    s = _solver(wl, max_targets=100)
    out = s.predict(dev(z), dev(wl.targets), PcgOptions())
    assert out["info"]["inner_iters"] == 0            # Z_W at rounding level: gamma_W = 0
    assert relerr(out["beta"], beta0) < 1e-10
    assert np.abs(host(out["gamma"])).max() < 1e-8
    np.testing.assert_allclose(host(out["zhat"]), design_matrix(wl.targets, wl.degree_w) @ beta0, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("prec", [1, 2, 3])
def test_mixed_precision_refinement_reaches_fp64_residual(prec, scheme):
    """Both mixed schemes (flexible CG around inner solves; one recurrence
    with reliable updates) reach the FP64 residual and the oracle."""
    torch = require_gpu()
    from paper_1701_00285_amd import FP64, PcgOptions
    wl = workload(4, n=3000, n_targets=300)
    s = _solver(wl, max_targets=300)
    say(f"mixed precision={prec} scheme={scheme}")
    a = s.predict(dev(wl.z), dev(wl.targets), PcgOptions(rtol=1e-8, precision=FP64, max_iter=5000))
    b = s.predict(dev(wl.z), dev(wl.targets), PcgOptions(rtol=1e-8, precision=prec, inner_rtol=1e-4,
                                                         max_iter=5000, mixed_scheme=scheme))
    assert b["info"]["relres_fp64"] <= 1e-8
    assert b["info"]["lowp_matvecs"] > 0
    ref = OB.classic_blup(wl.points, wl.z, wl.targets, wl.degree_w, wl.nu, wl.rho)
    assert relerr(host(b["zhat"]), ref.zhat) < 1e-6
    assert relerr(host(b["zhat"]), host(a["zhat"])) < 1e-6
    if scheme == 1:
        # one recurrence: a residual replacement per factor inner_rtol, not a restart
        assert b["info"]["fp64_matvecs"] <= b["info"]["outer_iters"] + 3


def test_reliable_update_keeps_the_recurrence():
    """Reliable updates replace the residual without restarting: the
    low-precision recurrence needs about as many iterations as FP64 PCG,
    and a cap on replacements ends the solve with ENOCONV."""
    torch = require_gpu()
    from paper_1701_00285_amd import FP32, FP64, MIXED_RELIABLE, PcgOptions
    from paper_1701_00285_amd import _lib as L
    wl = workload(3, n=4000, n_targets=10)
    s = _solver(wl)
    zw, _ = s.apply_W(s.to_tree(dev(wl.z)))
    g64, i64, _ = s.solve(zw, PcgOptions(rtol=1e-9, max_iter=5000))
    gr, ir, _ = s.solve(zw, PcgOptions(rtol=1e-9, max_iter=5000, precision=FP32, inner_rtol=1e-2,
                                       mixed_scheme=MIXED_RELIABLE))
    say(f"fp64 {i64} reliable {ir}")
    assert ir["relres_fp64"] <= 1e-9 and ir["outer_iters"] >= 3
    assert ir["inner_iters"] <= 1.25 * i64["inner_iters"] + 10
    assert relerr(host(gr), host(g64)) < 1e-6
    _, ic, st = s.solve(zw, PcgOptions(rtol=1e-9, max_iter=5000, precision=FP32, inner_rtol=1e-2, refine_max=2,
                                       mixed_scheme=MIXED_RELIABLE), allow_noconv=True)
    assert st == L.ENOCONV and ic["outer_iters"] == 2


def test_error_paths():
    torch = require_gpu()
    from paper_1701_00285_amd import MlblupError, PcgOptions
    from paper_1701_00285_amd import _lib as L
    wl = workload(1)
    s = _solver(wl, max_targets=10)
    out = s.predict(dev(wl.z), dev(wl.targets[:10]), PcgOptions(max_iter=1), allow_noconv=True)
    assert out["status"] == L.ENOCONV and out["info"]["inner_iters"] == 1
    z = wl.z.copy()
    z[5] = np.nan
    with pytest.raises(MlblupError, match="EINVAL"):
        s.predict(dev(z), None, PcgOptions())
    zw = torch.zeros(s.n - s.p, dtype=torch.float64, device="cuda")
    gw, info, st = s.solve(zw)
    assert st == 0 and float(torch.abs(gw).max()) == 0.0
    with pytest.raises(MlblupError, match="EINVAL"):
        s.solve(zw, PcgOptions(rtol=-1.0))
    with pytest.raises(MlblupError, match="EINVAL"):
        s.solve(zw, PcgOptions(precision=1, mixed_scheme=7))
    from paper_1701_00285_amd import cov_matvec
    with pytest.raises(MlblupError, match="EINVAL"):
        cov_matvec(dev(wl.points), dev(wl.points), dev(wl.z), 9.0, 0.1)   # nu out of (0, 8]


def test_basis_independence_of_iterations():
    """Unpreconditioned CG on C_W is invariant under an orthogonal change of
    W; leaf 32 and leaf 64 trees give the same iteration count."""
    torch = require_gpu()
    from paper_1701_00285_amd import PcgOptions
    wl = workload(4, n=2000, n_targets=10)
    it, hist = [], []
    for leaf in (32, 64):
        s = _solver(wl, leaf=leaf)
        zw, _ = s.apply_W(s.to_tree(dev(wl.z)))
        h = np.zeros(5000)
        _, info, _ = s.solve(zw, PcgOptions(rtol=1e-8, max_iter=5000, history=h))
        it.append(info["inner_iters"])
        hist.append(h[:info["inner_iters"]])
    k = min(len(hist[0]), len(hist[1]), 30)       # early residual histories agree to rounding
    np.testing.assert_allclose(hist[0][:k], hist[1][:k], rtol=1e-6)
    # over hundreds of iterations rounding (loss of orthogonality) lets the
    # two finite-precision runs drift apart slightly
    assert abs(it[0] - it[1]) <= 0.03 * max(it) + 2


@pytest.mark.parametrize("k,prec,scheme", [(5, 2, 0), (5, 3, 0), (3, 2, 0), (5, 2, 1), (3, 3, 1)])
def test_mixed_matrix_core_solve(k, prec, scheme):
    """Mixed solves whose inner products use the matrix-core distance Gram
    (d = 20 and d = 10 workloads, subsampled) reach the FP64 residual and
    the oracle's predictions."""
    torch = require_gpu()
    from paper_1701_00285_amd import PREC_BLOCK, PcgOptions
    wl = workload(k, n=3000, n_targets=200)
    say(f"mixed matrix-core cfg{k} precision={prec} scheme={scheme}")
    s = _solver(wl, max_targets=200)
    pc = s.precond(PREC_BLOCK)
    out = s.predict(dev(wl.z), dev(wl.targets), PcgOptions(rtol=1e-10, precision=prec, inner_rtol=1e-2,
                                                           precond=pc, max_iter=5000, mixed_scheme=scheme))
    assert out["info"]["relres_fp64"] <= 1e-10
    assert out["info"]["lowp_matvecs"] > 0
    ref = OB.classic_blup(wl.points, wl.z, wl.targets, wl.degree_w, wl.nu, wl.rho)
    assert relerr(host(out["zhat"]), ref.zhat) < 1e-8


@pytest.mark.parametrize("nu", [0.75, 1.0, 1.25])
def test_general_nu_blup_matches_oracle(nu):
    """The predictor with a general smoothness (FP64 products from the table)
    against the oracle's classic BLUP with scipy's K_nu."""
    torch = require_gpu()
    from paper_1701_00285_amd import PcgOptions
    wl = workload(4, n=2000, n_targets=150)
    say(f"general nu={nu} blup")
    s = _solver(wl, max_targets=150, nu=nu)
    out = s.predict(dev(wl.z), dev(wl.targets), PcgOptions(rtol=1e-12, max_iter=6000))
    ref = OB.classic_blup(wl.points, wl.z, wl.targets, wl.degree_w, nu, wl.rho)
    assert relerr(host(out["zhat"]), ref.zhat) < 1e-9
    assert relerr(out["beta"], ref.beta) < 1e-8


def test_general_nu_mixed_solve_gradient_and_preconditioner():
    """nu = 5/4 (the smoothness of the paper's prediction experiments) through
    the whole path: the block preconditioner built with FP32 general-nu
    values, the flexible-CG mixed solve with FP32 inner products, the FP64
    predictor, and Q, dQ/dlog rho from the general-nu derivative kernel;
    against the oracle's classic BLUP and dense gradient (scipy K_nu, K_{nu-1})."""
    torch = require_gpu()
    from paper_1701_00285_amd import FP32, FP64, PREC_BLOCK, PcgOptions
    nu = 1.25
    wl = workload(4, n=2000, n_targets=150)
    s = _solver(wl, max_targets=150, nu=nu)
    pc = s.precond(PREC_BLOCK)
    ref = OB.classic_blup(wl.points, wl.z, wl.targets, wl.degree_w, nu, wl.rho)
    q_ref, dq_ref = OB.quad_form_grad(wl.points, wl.z, wl.degree_w, nu, wl.rho)
    plain = s.predict(dev(wl.z), dev(wl.targets), PcgOptions(rtol=1e-12, max_iter=6000, precision=FP64))
    a = s.predict(dev(wl.z), dev(wl.targets), PcgOptions(rtol=1e-12, max_iter=6000, precision=FP64, precond=pc))
    b = s.predict(dev(wl.z), dev(wl.targets), PcgOptions(rtol=1e-8, max_iter=6000, precision=FP32, inner_rtol=0.1,
                                                         precond=pc))
    say(f"general nu={nu}: fp64 {plain['info']['inner_iters']} it (block: {a['info']['inner_iters']}), mixed "
        f"{b['info']['inner_iters']} inner / {b['info']['outer_iters']} outer, zhat err "
        f"{relerr(host(a['zhat']), ref.zhat):.2e} / {relerr(host(b['zhat']), ref.zhat):.2e}")
    assert a["info"]["inner_iters"] < plain["info"]["inner_iters"]
    assert relerr(host(a["zhat"]), ref.zhat) < 1e-9
    assert b["info"]["relres_fp64"] <= 1e-8 and b["info"]["lowp_matvecs"] > 0
    assert relerr(host(b["zhat"]), ref.zhat) < 1e-6
    zt = s.to_tree(dev(wl.z))
    q, dq = s.quad_grad(zt, a["gamma_tree"])
    say(f"general nu={nu}: Q {abs(q - q_ref) / abs(q_ref):.2e} dQ {abs(dq - dq_ref) / abs(dq_ref):.2e}")
    assert abs(q - q_ref) <= 1e-8 * abs(q_ref)
    assert abs(dq - dq_ref) <= 1e-8 * abs(dq_ref)


@pytest.mark.parametrize("precond", [None, "block"])
def test_fp64_solve_resumes_its_recurrence(precond):
    """Checkpoint / resume of the FP64 PCG: a solve stopped after half its
    iterations, with its Krylov state (r, p, r.z) kept, and continued from
    gamma_W with that state, takes exactly the iterations that remain in the
    uninterrupted solve and ends on the same gamma_W (up to the rounding of
    splitting the update of gamma_W in two); the result matches the oracle."""
    torch = require_gpu()
    from paper_1701_00285_amd import FP64, PREC_BLOCK, MlblupError, PcgOptions, Solver
    wl = workload(2, n=3000, n_targets=1)
    s = Solver(wl.points, wl.degree_w, wl.leaf_max, wl.nu, wl.rho, wl.sigma2)
    pc = s.precond(PREC_BLOCK) if precond else None
    zw, _ = s.apply_W(s.to_tree(dev(wl.z)))
    full, info_full, _ = s.solve(zw, PcgOptions(rtol=1e-10, max_iter=20000, precision=FP64, precond=pc))
    n_full = info_full["inner_iters"]
    half = n_full // 2
    state = torch.empty(2 * (s.n - s.p) + 8, dtype=torch.float64, device="cuda")
    g1, info1, st1 = s.solve(zw, PcgOptions(rtol=1e-10, max_iter=half, precision=FP64, precond=pc, state=state),
                             allow_noconv=True)
    assert st1 != 0 and info1["inner_iters"] == half
    g2, info2, st2 = s.solve(zw, PcgOptions(rtol=1e-10, max_iter=20000, precision=FP64, precond=pc, state=state,
                                            resume=True), x0=g1)
    say(f"resume ({precond}): uninterrupted {n_full} iterations, segments {half} + {info2['inner_iters']}, "
        f"relres {info2['relres_fp64']:.2e}")
    assert st2 == 0 and info2["relres_fp64"] <= 1e-10
    assert half + info2["inner_iters"] == n_full
    assert float(torch.linalg.norm(g2 - full) / torch.linalg.norm(full)) < 1e-9
    with pytest.raises(MlblupError):
        s.solve(zw, PcgOptions(rtol=1e-10, max_iter=10, precision=FP64, state=state, resume=True))  # no x0


def test_trend_of_351_terms_d25():
    """The paper's largest-p setting class: d = 25, total degree 2 (p = 351
    trend terms).  Leaves of up to 128 points hold no wavelets (s <= p, all
    scaling), internal cells up to 702 candidates: the transform takes its
    reflector chain (leaves) and dense-block (m > 256) paths.  FP64 predict
    against the oracle's dense classic BLUP."""
    torch = require_gpu()
    from paper_1701_00285_amd import FP64, PcgOptions, Solver
    n, d, nt = 1500, 25, 40
    pts = synth.uniform_cloud(n, d, 2501)
    tgt = synth.uniform_cloud(nt, d, 2502)
    z = np.sin(3.0 * pts[:, 0]) + pts[:, 1] * pts[:, 2] + 0.3 * synth.standard_normal(n, 2503)
    ref = OB.classic_blup(pts, z, tgt, 2, 0.5, 2.0)
    s = Solver(pts, 2, 128, 0.5, 2.0, 1.0, max_targets=nt)
    assert s.p == 351
    say(f"p=351 d=25 n={n}: levels {s.basis.levels}, transform bytes {s.basis.transform_bytes()}")
    out = s.predict(dev(z), dev(tgt), PcgOptions(rtol=1e-12, max_iter=4000, precision=FP64))
    assert out["info"]["relres_fp64"] <= 1e-12
    assert relerr(host(out["zhat"]), ref.zhat) < 1e-8
    assert relerr(host(out["gamma"]), ref.gamma) < 1e-8
