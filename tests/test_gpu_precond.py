"""Preconditioner P_W (diag(C_W) and its per-cell blocks) built on the GPU
against C_W formed densely from the oracle's covariance, and the
preconditioned solve against the unpreconditioned one."""
import numpy as np
import pytest

from gpu_common import dev, host, require_gpu, say
from helpers import relerr, workload
from oracle.basis import build_basis
from oracle.kdtree import build_kdtree
from oracle.matern import cov_matrix

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k,n", [(1, 1000), (2, 1500), (4, 1200), (3, 1100), (5, 900)])
def test_blocks_match_dense_cw(k, n):
    torch = require_gpu()
    from paper_1701_00285_amd import PREC_BLOCK, PREC_JACOBI, Solver
    wl = workload(k, n=n, n_targets=1)
    say(f"precond blocks cfg{k} n={n}")
    s = Solver(wl.points, wl.degree_w, wl.leaf_max, wl.nu, wl.rho)
    pc = s.precond(PREC_BLOCK)
    W, _ = s.basis.dense()
    pts_t = wl.points[s.tree.perm]
    CW = W @ cov_matrix(pts_t, pts_t, wl.nu, wl.rho) @ W.T
    blocks, woff = pc.blocks()
    assert sum(b.shape[0] for b in blocks) == n - s.p
    scale = np.abs(np.diag(CW)).max()
    for B, o in zip(blocks, woff):
        m = B.shape[0]
        ref = CW[o:o + m, o:o + m]
        assert np.abs(B - ref).max() <= 2e-6 * max(np.abs(ref).max(), 1e-3 * scale)
    # basis-independent pin: each block's spectrum equals that of the same
    # cell's block in the oracle's SVD basis
    ob = build_basis(wl.points, build_kdtree(wl.points, wl.leaf_max), wl.degree_w)
    Co = cov_matrix(wl.points, wl.points, wl.nu, wl.rho)
    rows = sorted(ob.node_rows.values())
    rows = [r for r in rows if r[1] > 0]
    assert len(rows) == len(blocks)
    for (off, cnt), B in zip(rows, blocks):
        Wv = ob.W[off:off + cnt]
        ev_o = np.linalg.eigvalsh(Wv @ Co @ Wv.T)
        ev_c = np.linalg.eigvalsh(B)
        np.testing.assert_allclose(ev_c, ev_o, atol=2e-6 * max(ev_o.max(), 1e-3 * scale))
    pj = s.precond(PREC_JACOBI)
    bj, _ = pj.blocks()
    for a, b in zip(bj, blocks):
        np.testing.assert_array_equal(np.diag(a), np.diag(b))


@pytest.mark.parametrize("k,n", [(2, 3000), (4, 3000)])
def test_preconditioned_solves_agree_and_converge_faster(k, n):
    torch = require_gpu()
    from paper_1701_00285_amd import PREC_BLOCK, PREC_JACOBI, PcgOptions, Solver
    wl = workload(k, n=n, n_targets=1)
    say(f"preconditioned solve cfg{k} n={n}")
    s = Solver(wl.points, wl.degree_w, wl.leaf_max, wl.nu, wl.rho)
    zw, _ = s.apply_W(s.to_tree(dev(wl.z)))
    res = {}
    for name, kind in (("none", None), ("jacobi", PREC_JACOBI), ("block", PREC_BLOCK)):
        pc = s.precond(kind) if kind else None
        gw, info, st = s.solve(zw, PcgOptions(rtol=1e-10, max_iter=20000, precond=pc))
        assert st == 0 and info["relres_fp64"] <= 1e-10
        res[name] = (host(gw), info["inner_iters"])
    assert relerr(res["jacobi"][0], res["none"][0]) < 1e-6
    assert relerr(res["block"][0], res["none"][0]) < 1e-6
    assert res["block"][1] < res["none"][1]
    assert res["jacobi"][1] < res["none"][1]
