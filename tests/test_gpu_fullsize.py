"""End-to-end parity at the sizes where the solve takes the kernels of the
full-size workloads: the symmetric pair kernels (FP64 and FP32 direct, and
the matrix-core rounds kernel in FP32 and BF16 x3) switch on at 16,384
points, so every case here has n >= 16,384, with odd block counts and
ragged last blocks where the size allows.  Each case goes through
Solver.predict / quad_grad (the C ABI) with the preconditioner and the
mixed-precision scheme its workload uses in the bench, and is compared
element by element with the oracle's dense classic BLUP (Sec. 2 eqs.
GLSbeta / KrigBLUP; Sec. 5.2 eqs. Spatial:eqn1-3 give the same values) and
its dense gradient.

Tolerances.  FP64 path: solved to relres 1e-12, predictions and beta-hat
within 1e-10 and gamma-hat within 1e-9 of the oracle, as the small-size FP64
parity tests.  Mixed path: solved to the bench's relres 1e-8; the north-star
bar for predictions is 1e-6 relative, and beta-hat follows from the same
residual (L v).  gamma-hat itself is only as good as relres times the
condition of C_W, so it is checked at the looser 1e-4 (the predictions are
the quantity of interest).  Gradient: Q and dQ/dlog rho within 1e-8 of the
dense oracle gradient after an FP64 solve to 1e-12; the mixed path to 1e-10
within 1e-7."""
import numpy as np
import pytest

from gpu_common import dev, host, require_gpu, say
from helpers import workload
from oracle import blup as OB

pytestmark = pytest.mark.gpu

_ORACLE = {}


def _oracle(k, n, nt):
    key = (k, n, nt)
    if key not in _ORACLE:
        wl = workload(k, n=n, n_targets=nt)
        say(f"oracle: dense classic BLUP, workload {k} generator, n={n}, {nt} targets")
        _ORACLE[key] = (wl, OB.classic_blup(wl.points, wl.z, wl.targets, wl.degree_w, wl.nu, wl.rho))
    return _ORACLE[key]


def _maxrel(a, b):
    """max_i |a_i - b_i| / max_i |b_i| (element-wise, scaled by the largest entry)."""
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _check(out, ref, tz, tb, tg, label):
    ez = _maxrel(host(out["zhat"]), ref.zhat)
    eb = _maxrel(out["beta"], ref.beta)
    eg = _maxrel(host(out["gamma"]), ref.gamma)
    say(f"{label}: iters {out['info']['inner_iters']} outer {out['info']['outer_iters']} "
        f"relres {out['info']['relres_fp64']:.2e}  zhat {ez:.2e} beta {eb:.2e} gamma {eg:.2e}")
    assert ez < tz and eb < tb and eg < tg, (label, ez, eb, eg)


def _solver(wl, nt):
    from paper_1701_00285_amd import Solver
    return Solver(wl.points, wl.degree_w, wl.leaf_max, wl.nu, wl.rho, wl.sigma2, max_targets=nt)


def test_fullsize_d3_coarse_preconditioner_fp64_and_mixed():
    """Workload 2 generator at 17,000 points (17 blocks of 1,024: odd
    tournament, ragged last block): the coarse preconditioner, the FP64
    symmetric kernel, and the flexible-CG mixed solve with the FP32
    symmetric kernel (inner tolerance 0.35, as in the bench)."""
    require_gpu()
    from paper_1701_00285_amd import FP32, FP64, PREC_COARSE, PcgOptions
    wl, ref = _oracle(2, 17000, 2048)
    s = _solver(wl, 2048)
    pc = s.precond(PREC_COARSE)
    z, t = dev(wl.z), dev(wl.targets)
    a = s.predict(z, t, PcgOptions(rtol=1e-12, max_iter=20000, precision=FP64, precond=pc))
    assert a["info"]["relres_fp64"] <= 1e-12
    _check(a, ref, 1e-10, 1e-10, 1e-9, "d=3 coarse fp64")
    b = s.predict(z, t, PcgOptions(rtol=1e-8, max_iter=20000, precision=FP32, inner_rtol=0.35, precond=pc))
    assert b["info"]["relres_fp64"] <= 1e-8 and b["info"]["lowp_matvecs"] > 0
    _check(b, ref, 1e-6, 1e-6, 1e-4, "d=3 coarse mixed fp32")


@pytest.mark.parametrize("prec", [2, 3])
def test_fullsize_d10_matrix_core_mixed(prec):
    """Workload 3 generator (8 clusters in d = 10) at 16,384 points: the FP64
    symmetric kernel (blocks of 512: 32 blocks) and the mixed solve whose
    inner products run the matrix-core rounds kernel (FP32 or BF16 x3
    Gram); P_W = I as in the full-size runs."""
    require_gpu()
    from paper_1701_00285_amd import FP64, PcgOptions
    wl, ref = _oracle(3, 16384, 2048)
    s = _solver(wl, 2048)
    z, t = dev(wl.z), dev(wl.targets)
    if prec == 2:
        a = s.predict(z, t, PcgOptions(rtol=1e-12, max_iter=20000, precision=FP64))
        _check(a, ref, 1e-10, 1e-10, 1e-9, "d=10 fp64")
    b = s.predict(z, t, PcgOptions(rtol=1e-8, max_iter=20000, precision=prec, inner_rtol=0.1))
    assert b["info"]["relres_fp64"] <= 1e-8 and b["info"]["lowp_matvecs"] > 0
    _check(b, ref, 1e-6, 1e-6, 1e-4, f"d=10 mixed precision {prec}")


def test_fullsize_d20_matrix_core_mixed():
    """Workload 5 generator (d = 20, half uniform, half near a 3-d subspace)
    at 16,700 points (33 blocks of 512, ragged last block): FP64 symmetric
    kernel and the BF16 x3 matrix-core mixed solve, P_W = I."""
    require_gpu()
    from paper_1701_00285_amd import FP64, MFMA_BF16X3, PcgOptions
    wl, ref = _oracle(5, 16700, 2048)
    s = _solver(wl, 2048)
    z, t = dev(wl.z), dev(wl.targets)
    a = s.predict(z, t, PcgOptions(rtol=1e-12, max_iter=20000, precision=FP64))
    _check(a, ref, 1e-10, 1e-10, 1e-9, "d=20 fp64")
    b = s.predict(z, t, PcgOptions(rtol=1e-8, max_iter=20000, precision=MFMA_BF16X3, inner_rtol=0.1))
    assert b["info"]["relres_fp64"] <= 1e-8 and b["info"]["lowp_matvecs"] > 0
    _check(b, ref, 1e-6, 1e-6, 1e-4, "d=20 mixed bf16x3")


def test_fullsize_d5_gradient():
    """Workload 4 generator at 16,384 points (nu = 5/2, d = 5): Q and
    dQ/dlog rho through the symmetric derivative kernel, after the
    coarse-preconditioned FP64 solve and the FP32 mixed solve, against the
    dense oracle gradient."""
    require_gpu()
    from paper_1701_00285_amd import FP32, FP64, PREC_COARSE, PcgOptions
    wl = workload(4, n=16384, n_targets=1)
    say("oracle: dense gradient, workload 4 generator, n=16384")
    Q0, dQ0 = OB.quad_form_grad(wl.points, wl.z, wl.degree_w, wl.nu, wl.rho)
    s = _solver(wl, 0)
    pc = s.precond(PREC_COARSE)
    zt = s.to_tree(dev(wl.z))
    zw, _ = s.apply_W(zt)
    for prec, rtol, tol in ((FP64, 1e-12, 1e-8), (FP32, 1e-10, 1e-7)):
        gw, info, _ = s.solve(zw, PcgOptions(rtol=rtol, max_iter=20000, precision=prec, inner_rtol=0.35, precond=pc))
        q, dq = s.quad_grad(zt, s.apply_Wt(gw))
        say(f"d=5 gradient precision {prec}: iters {info['inner_iters']} Q {abs(q - Q0) / abs(Q0):.2e} "
            f"dQ {abs(dq - dQ0) / abs(dQ0):.2e}")
        assert abs(q - Q0) <= tol * abs(Q0)
        assert abs(dq - dQ0) <= tol * abs(dQ0)
