"""Multilevel log-likelihood and its maximum in rho on the GPU against the
oracle (dense C^n_W from the oracle's SVD basis, numpy Cholesky).  The two
bases differ by rotations inside the cells, under which l_n is invariant."""
import math

import numpy as np
import pytest

from gpu_common import dev, require_gpu, say
from helpers import workload
from oracle import likelihood as OL
from oracle.basis import build_basis
from oracle.kdtree import build_kdtree
from oracle.matern import cov_matrix

pytestmark = pytest.mark.gpu


def _both(k, n, nu=None):
    from paper_1701_00285_amd import Solver
    wl = workload(k, n=n, n_targets=1)
    nu = wl.nu if nu is None else nu
    tree = build_kdtree(wl.points, wl.leaf_max)
    bas = build_basis(wl.points, tree, wl.degree_w)
    s = Solver(wl.points, wl.degree_w, wl.leaf_max, nu, wl.rho, wl.sigma2)
    return wl, nu, tree, bas, s


def _cond(wl, nu, bas, nt):
    C = cov_matrix(wl.points, wl.points, nu, wl.rho)
    ev = np.linalg.eigvalsh(bas.W[:nt] @ C @ bas.W[:nt].T)
    return ev[-1] / ev[0]


@pytest.mark.parametrize("k,n,nu", [(1, 1000, None), (2, 900, None), (4, 700, None), (2, 650, 1.25), (1, 777, 1.5)])
def test_loglik_matches_oracle(k, n, nu):
    require_gpu()
    wl, nu, tree, bas, s = _both(k, n, nu)
    Z = dev(wl.z)
    t = tree.max_depth
    for level in sorted({t, t - 1, 1, 0}, reverse=True):
        g = s.loglik(Z, level)
        o = OL.multilevel_loglik(wl.points, wl.z, nu, wl.rho, bas, level)
        kap = _cond(wl, nu, bas, o[3])
        # backward-stable factorizations of C^n_W from two bases: errors of
        # order kappa u in the quadratic form, N~ kappa u in log det (absolute)
        tq = max(1e-12, 50 * kap * 2.2e-16)
        td = max(1e-12, 50 * kap * 2.2e-16) * o[3]
        say(f"loglik cfg{k} n={n} nu={nu} level={level} rows={g['rows']} kappa={kap:.1e} "
            f"dlogdet={abs(g['logdet'] - o[1]):.1e} dquad={abs(g['quad'] - o[2]) / abs(o[2]):.1e}")
        assert g["rows"] == o[3]
        assert abs(g["logdet"] - o[1]) < td
        assert abs(g["quad"] - o[2]) < tq * abs(o[2])
        assert abs(g["loglik"] - o[0]) < td + tq * abs(o[2])


def test_level0_quadratic_form_is_the_solve_Q():
    """At level 0 the quadratic form is Z_W^T C_W^-1 Z_W, the Q of the PCG path."""
    torch = require_gpu()
    from paper_1701_00285_amd import FP64, PcgOptions
    wl, nu, tree, bas, s = _both(2, 800)
    Z = dev(wl.z)
    g = s.loglik(Z, 0)
    out = s.predict(Z, None, PcgOptions(rtol=1e-13, max_iter=5000, precision=FP64))
    q = float(torch.dot(Z, out["gamma"]))
    assert abs(g["quad"] - q) < 1e-8 * abs(q)


def test_mle_rho_matches_oracle():
    require_gpu()
    wl, nu, tree, bas, s = _both(1, 600)
    Z = dev(wl.z)
    level = tree.max_depth - 1
    g = s.mle_rho(Z, level, 0.01, 1.0, 1e-5)
    o = OL.mle_rho(wl.points, wl.z, nu, bas, level, 0.01, 1.0, 1e-5)
    say(f"mle rho gpu {g['rho']:.8f} oracle {o[0]:.8f} evals {g['evals']}")
    assert abs(math.log(g["rho"]) - math.log(o[0])) < 3e-5
    assert abs(g["loglik"] - o[1]) < 1e-9 * abs(o[1])
    assert g["bracket"] <= 1e-5


def test_loglik_error_paths():
    torch = require_gpu()
    import ctypes as C
    from paper_1701_00285_amd import MlblupError, matern
    from paper_1701_00285_amd import _lib as L
    wl, nu, tree, bas, s = _both(1, 300)
    with pytest.raises(MlblupError, match="EINVAL"):
        s.loglik(dev(wl.z), s.basis.levels)
    k = matern(nu, wl.rho)
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    out = np.zeros(4)
    zt = s.to_tree(dev(wl.z)).contiguous()
    st = L.lib().mlblup_loglik(s.basis.h, C.byref(k), C.c_void_p(zt.data_ptr()), 0, math.inf,
                               out.ctypes.data_as(C.c_void_p), C.c_void_p(small.data_ptr()), small.numel(), None)
    assert st == L.EINVAL
    with pytest.raises(MlblupError, match="EINVAL"):
        s.mle_rho(dev(wl.z), 0, 1.0, 0.5)
    for tau in (-0.5, float("nan")):
        with pytest.raises(MlblupError, match="EINVAL"):
            s.loglik(dev(wl.z), 0, tau=tau)


def test_mle_nu_rho_matches_oracle():
    """Profile-likelihood MLE of (nu, rho): golden section over nu with the
    rho maximum at each point, on the GPU (general-nu FP64 kernel values) and
    in the oracle (Bessel-form covariance)."""
    require_gpu()
    wl, nu, tree, bas, s = _both(1, 300)
    Z = dev(wl.z)
    level = tree.max_depth - 1
    g = s.mle_nu_rho(Z, level, 0.3, 2.0, 0.02, 0.5, nu_tol=1e-2, log_rho_tol=1e-3)
    o = OL.mle_nu_rho(wl.points, wl.z, bas, level, 0.3, 2.0, 0.02, 0.5, 1e-2, 1e-3)
    say(f"mle (nu, rho) gpu ({g['nu']:.5f}, {g['rho']:.5f}) oracle ({o[0]:.5f}, {o[1]:.5f}) evals {g['evals']}")
    assert abs(g["nu"] - o[0]) < 2e-2
    assert abs(math.log(g["rho"]) - math.log(o[1])) < 5e-3
    assert abs(g["loglik"] - o[2]) < 1e-8 * abs(o[2])


# ---- sparsified C~^n_W (Sec. 4.1 tree search with distance tau) ------------------

def _cond_sparse(wl, nu, tree, bas, level, tau):
    nt = OL.level_rows(bas, level)
    C = cov_matrix(wl.points, wl.points, nu, wl.rho)
    Cn = bas.W[:nt] @ C @ bas.W[:nt].T
    ev = np.linalg.eigvalsh(np.where(OL.sparsity_mask(wl.points, tree, bas, level, tau), Cn, 0.0))
    return ev[-1] / ev[0]


# (cfg, n, levels below the finest, tau): cases where C~^n_W stays positive definite
SPARSE = [(1, 1000, 0, 0.0), (1, 1000, 0, 0.05), (1, 1000, 1, 0.05), (1, 1000, 1, 0.2),
          (2, 900, 0, 0.0), (2, 900, 0, 0.05), (2, 900, 1, 0.1), (4, 700, 0, 0.0), (4, 700, 1, 0.2)]


@pytest.mark.parametrize("k,n,up,tau", SPARSE)
def test_sparsified_loglik_matches_oracle(k, n, up, tau):
    require_gpu()
    wl, nu, tree, bas, s = _both(k, n)
    level = tree.max_depth - up
    g = s.loglik(dev(wl.z), level, tau=tau)
    o = OL.multilevel_loglik(wl.points, wl.z, nu, wl.rho, bas, level, tree=tree, tau=tau)
    kap = _cond_sparse(wl, nu, tree, bas, level, tau)
    assert kap > 0
    tq = max(1e-12, 50 * kap * 2.2e-16)
    td = tq * o[3]
    say(f"sparse loglik cfg{k} n={n} level={level} tau={tau} nnz={g['nnz']} kappa={kap:.1e} "
        f"dlogdet={abs(g['logdet'] - o[1]):.1e} dquad={abs(g['quad'] - o[2]) / abs(o[2]):.1e}")
    assert g["nnz"] == s.basis.sparsity_pattern(level, tau) == int(
        OL.sparsity_mask(wl.points, tree, bas, level, tau).sum())
    assert abs(g["logdet"] - o[1]) < td
    assert abs(g["quad"] - o[2]) < tq * abs(o[2])
    assert abs(g["loglik"] - o[0]) < td + tq * abs(o[2])


def test_sparsified_loglik_with_everything_kept_is_the_exact_value():
    require_gpu()
    wl, nu, tree, bas, s = _both(2, 900)
    z = dev(wl.z)
    for level in (tree.max_depth, 1):
        a = s.loglik(z, level)
        b = s.loglik(z, level, tau=4.0)   # the widened unit cube covers every region
        assert a["nnz"] == b["nnz"] == a["rows"] ** 2
        assert (a["loglik"], a["logdet"], a["quad"]) == (b["loglik"], b["logdet"], b["quad"])


@pytest.mark.parametrize("k,n,level,tau", [(1, 1000, 0, 0.0), (4, 700, -1, 0.02)])
def test_indefinite_sparsified_matrix_is_a_breakdown(k, n, level, tau):
    """Small tau at coarse levels drops enough of C^n_W to make it indefinite
    (smallest eigenvalue about -0.2 and -0.1 here): EBREAKDOWN, as the
    oracle's Cholesky fails too."""
    require_gpu()
    from paper_1701_00285_amd import MlblupError
    wl, nu, tree, bas, s = _both(k, n)
    level = tree.max_depth if level < 0 else level
    with pytest.raises(np.linalg.LinAlgError):
        OL.multilevel_loglik(wl.points, wl.z, nu, wl.rho, bas, level, tree=tree, tau=tau)
    with pytest.raises(MlblupError, match="EBREAKDOWN"):
        s.loglik(dev(wl.z), level, tau=tau)
    # the workspace stays usable
    g = s.loglik(dev(wl.z), tree.max_depth, tau=0.0 if k == 1 else 0.2)
    assert math.isfinite(g["loglik"])


def test_sparsified_mle_rho_matches_oracle():
    require_gpu()
    wl, nu, tree, bas, s = _both(1, 600)
    level = tree.max_depth - 1
    g = s.mle_rho(dev(wl.z), level, 0.01, 1.0, 1e-5, tau=0.05)
    o = OL.mle_rho(wl.points, wl.z, nu, bas, level, 0.01, 1.0, 1e-5, tree=tree, tau=0.05)
    say(f"sparse mle rho gpu {g['rho']:.8f} oracle {o[0]:.8f} evals {g['evals']}")
    assert abs(math.log(g["rho"]) - math.log(o[0])) < 3e-5
    assert abs(g["loglik"] - o[1]) < 1e-9 * abs(o[1])


@pytest.mark.parametrize("n", [67, 68, 131, 259, 260, 387, 515, 771])
def test_loglik_at_block_and_panel_boundaries(n):
    """Level 0 of the d = 2 linear-trend workload has N~ = n - 3 rows: 64, 65,
    128, 256, 257, 384, 512 and 768 put the end of the matrix (and the border
    row that carries Z^n_W) exactly on, or one past, the 64-column blocks, the
    128-row update tiles and the 256-column panels."""
    require_gpu()
    wl, nu, tree, bas, s = _both(1, n)
    g = s.loglik(dev(wl.z), 0)
    o = OL.multilevel_loglik(wl.points, wl.z, nu, wl.rho, bas, 0)
    assert g["rows"] == o[3] == n - 3
    kap = _cond(wl, nu, bas, o[3])
    tq = max(1e-12, 50 * kap * 2.2e-16)
    say(f"loglik boundary n={n} rows={o[3]} kappa={kap:.1e} dlogdet={abs(g['logdet'] - o[1]):.1e}")
    assert abs(g["logdet"] - o[1]) < tq * o[3]
    assert abs(g["quad"] - o[2]) < tq * abs(o[2])


def test_sparsified_mle_nu_rho_matches_oracle():
    """Profile MLE of (nu, rho) on the sparsified likelihood (tau = 0.05,
    the finest level, where C~ stays positive definite over the search box)."""
    require_gpu()
    wl, nu, tree, bas, s = _both(1, 300)
    level = tree.max_depth
    g = s.mle_nu_rho(dev(wl.z), level, 0.3, 2.0, 0.02, 0.5, nu_tol=1e-2, log_rho_tol=1e-3, tau=0.05)
    o = OL.mle_nu_rho(wl.points, wl.z, bas, level, 0.3, 2.0, 0.02, 0.5, 1e-2, 1e-3, tree=tree, tau=0.05)
    say(f"sparse mle (nu, rho) gpu ({g['nu']:.5f}, {g['rho']:.5f}) oracle ({o[0]:.5f}, {o[1]:.5f})")
    assert abs(g["nu"] - o[0]) < 2e-2
    assert abs(math.log(g["rho"]) - math.log(o[1])) < 5e-3
    assert abs(g["loglik"] - o[2]) < 1e-8 * abs(o[2])


# ---- sparse block factorization of C~^n_W (only the kept blocks are formed) --------

@pytest.mark.parametrize("k,n,up,tau,nu", [c + (None,) for c in SPARSE] + [(2, 650, 0, 0.05, 1.25),
                                                                          (2, 650, 1, 0.1, 1.25)])
def test_sparse_factorization_matches_oracle(k, n, up, tau, nu):
    """l~_n from the kept blocks and a block Cholesky over the cells equals
    the oracle's dense sparsified l~_n (same kappa-scaled tolerance as the
    dense path) and the dense GPU path on the same matrix."""
    require_gpu()
    wl, nu, tree, bas, s = _both(k, n, nu)
    level = tree.max_depth - up
    g = s.loglik_sparse(dev(wl.z), level, tau)
    d = s.loglik(dev(wl.z), level, tau=tau)
    o = OL.multilevel_loglik(wl.points, wl.z, nu, wl.rho, bas, level, tree=tree, tau=tau)
    kap = _cond_sparse(wl, nu, tree, bas, level, tau)
    tq = max(1e-12, 50 * kap * 2.2e-16)
    td = tq * o[3]
    info = s.loglik_sparse_info(level, tau)
    say(f"sparse factor cfg{k} n={n} nu={nu} level={level} tau={tau} rows={g['rows']} nnz={g['nnz']} "
        f"factor={info['factor_entries']} heights={info['heights']} kappa={kap:.1e} "
        f"dlogdet={abs(g['logdet'] - o[1]):.1e} dquad={abs(g['quad'] - o[2]) / abs(o[2]):.1e}")
    assert g["rows"] == o[3] == info["rows"]
    assert g["nnz"] == d["nnz"] == info["kept"]
    assert info["factor_entries"] >= info["kept"] // 2
    for ref in ((o[0], o[1], o[2]), (d["loglik"], d["logdet"], d["quad"])):
        assert abs(g["logdet"] - ref[1]) < td
        assert abs(g["quad"] - ref[2]) < tq * abs(ref[2])
        assert abs(g["loglik"] - ref[0]) < td + tq * abs(ref[2])


def test_sparse_factorization_everything_kept_and_repeated_calls():
    """tau beyond the domain keeps every block: the block factorization then
    gives the exact l_n; a second call with the same (level, tau) reuses the
    analysis and returns the same bits; another tau is analysed anew."""
    require_gpu()
    wl, nu, tree, bas, s = _both(2, 900)
    z = dev(wl.z)
    level = tree.max_depth - 1
    a = s.loglik(z, level)
    b = s.loglik_sparse(z, level, 4.0)
    kap = _cond(wl, nu, bas, a["rows"])
    tq = max(1e-12, 50 * kap * 2.2e-16)
    assert b["nnz"] == a["rows"] ** 2
    assert abs(a["logdet"] - b["logdet"]) < tq * a["rows"]
    assert abs(a["quad"] - b["quad"]) < tq * abs(a["quad"])
    c = s.loglik_sparse(z, level, 4.0)
    assert (b["loglik"], b["logdet"], b["quad"]) == (c["loglik"], c["logdet"], c["quad"])
    e = s.loglik_sparse(z, level, 0.1)
    f = s.loglik(z, level, tau=0.1)
    assert e["nnz"] == f["nnz"] < b["nnz"]
    assert abs(e["loglik"] - f["loglik"]) < 1e-9 * abs(f["loglik"])


@pytest.mark.parametrize("k,n,level,tau", [(1, 1000, 0, 0.0), (4, 700, -1, 0.02)])
def test_sparse_factorization_breakdown(k, n, level, tau):
    """The indefinite sparsified matrices of the dense test stop the block
    factorization too (EBREAKDOWN), and the next call works."""
    require_gpu()
    from paper_1701_00285_amd import MlblupError
    wl, nu, tree, bas, s = _both(k, n)
    level = tree.max_depth if level < 0 else level
    with pytest.raises(MlblupError, match="EBREAKDOWN"):
        s.loglik_sparse(dev(wl.z), level, tau)
    g = s.loglik_sparse(dev(wl.z), tree.max_depth, 0.0 if k == 1 else 0.2)
    assert math.isfinite(g["loglik"])


def test_sparse_factorization_rejects_large_cells():
    """A cell with more than 64 wavelets (leaves of 125 points, 115 wavelets
    each) is refused."""
    require_gpu()
    from paper_1701_00285_amd import MlblupError, Solver
    wl = workload(2, n=1000, n_targets=1)
    s = Solver(wl.points, wl.degree_w, 128, wl.nu, wl.rho, wl.sigma2)
    with pytest.raises(MlblupError, match="EINVAL"):
        s.loglik_sparse(dev(wl.z), 0, 0.05)


@pytest.mark.parametrize("up", [0, 1])
def test_sparse_factorization_at_16384_points(up):
    """16,384 points of the d = 3 workload's generator, against the dense
    GPU factorization of the same C~^n_W (sizes the oracle's eigenvalues
    cannot reach in seconds), for rough and smooth kernels and several tau:
    where the dense factorization finds C~^n_W indefinite the block one must
    too, elsewhere the two agree; rough kernels keep it definite."""
    require_gpu()
    from paper_1701_00285_amd import MlblupError, Solver
    wl = workload(2, n=16384, n_targets=1)
    z = dev(wl.z)
    compared = 0
    for nu, rho, tau in ((0.5, 0.02, 0.02), (0.5, 0.02, 0.05), (0.5, 0.05, 0.05), (1.5, 0.2, 0.05)):
        s = Solver(wl.points, wl.degree_w, wl.leaf_max, nu, rho, wl.sigma2)
        level = s.basis.levels - 1 - up
        try:
            d = s.loglik(z, level, tau=tau)
        except MlblupError as e:
            assert "EBREAKDOWN" in str(e)
            with pytest.raises(MlblupError, match="EBREAKDOWN"):
                s.loglik_sparse(z, level, tau)
            say(f"sparse factor 16384 nu={nu} rho={rho} level={level} tau={tau}: indefinite (both)")
            continue
        g = s.loglik_sparse(z, level, tau)
        info = s.loglik_sparse_info(level, tau)
        say(f"sparse factor 16384 nu={nu} rho={rho} level={level} tau={tau} rows={g['rows']} kept={g['nnz']} "
            f"factor={info['factor_entries']} heights={info['heights']} logdet {g['logdet']:.10e} / "
            f"{d['logdet']:.10e} quad {g['quad']:.10e} / {d['quad']:.10e}")
        assert g["nnz"] == d["nnz"]
        assert abs(g["logdet"] - d["logdet"]) < 1e-9 * g["rows"]
        assert abs(g["quad"] - d["quad"]) < 1e-8 * abs(d["quad"])
        compared += 1
    assert compared >= 1


def test_sparse_factorization_mle_rho_and_nu_rho():
    """The golden-section MLEs with every l~ evaluation by the block
    factorization: the rho MLE against the oracle's (tau = 0.05, level
    t - 1, as in the dense test), the profile (nu, rho) MLE against the dense
    GPU path's on the same sparsified likelihood (general-nu values)."""
    require_gpu()
    wl, nu, tree, bas, s = _both(1, 600)
    level = tree.max_depth - 1
    g = s.mle_rho(dev(wl.z), level, 0.01, 1.0, 1e-5, tau=0.05, sparse=True)
    o = OL.mle_rho(wl.points, wl.z, nu, bas, level, 0.01, 1.0, 1e-5, tree=tree, tau=0.05)
    say(f"sparse-factor mle rho gpu {g['rho']:.8f} oracle {o[0]:.8f} evals {g['evals']}")
    assert abs(math.log(g["rho"]) - math.log(o[0])) < 3e-5
    assert abs(g["loglik"] - o[1]) < 1e-9 * abs(o[1])
    wl, nu, tree, bas, s = _both(1, 300)
    level = tree.max_depth
    a = s.mle_nu_rho(dev(wl.z), level, 0.3, 2.0, 0.02, 0.5, nu_tol=1e-2, log_rho_tol=1e-3, tau=0.05, sparse=True)
    b = s.mle_nu_rho(dev(wl.z), level, 0.3, 2.0, 0.02, 0.5, nu_tol=1e-2, log_rho_tol=1e-3, tau=0.05)
    say(f"sparse-factor mle (nu, rho) ({a['nu']:.6f}, {a['rho']:.6f}) dense ({b['nu']:.6f}, {b['rho']:.6f})")
    assert a["evals"] == b["evals"]
    assert abs(a["nu"] - b["nu"]) < 1e-6 and abs(math.log(a["rho"]) - math.log(b["rho"])) < 1e-6
    assert abs(a["loglik"] - b["loglik"]) < 1e-9 * abs(b["loglik"])


@pytest.mark.parametrize("mode", ["none", "all", "auto", "cap128"])
@pytest.mark.parametrize("k,n,up,tau,nu", [(1, 1000, 0, 0.05, None), (2, 900, 1, 0.1, None), (4, 700, 1, 0.2, None),
                                            (2, 650, 0, 0.05, 1.25)])
def test_sparse_factorization_dense_tail_modes(monkeypatch, mode, k, n, up, tau, nu):
    """The block factorization with no dense tail, with all of C~^n_W as the
    dense tail (the block columns only assemble it), with the tail the
    analysis picks, and with that choice limited to 128 rows: the same l~ as
    the dense path on the same matrix."""
    require_gpu()
    monkeypatch.delenv("MLBLUP_SPARSE_TAIL_MAX", raising=False)
    if mode in ("auto", "cap128"):
        monkeypatch.delenv("MLBLUP_SPARSE_TAIL", raising=False)
        if mode == "cap128":
            monkeypatch.setenv("MLBLUP_SPARSE_TAIL_MAX", "128")
    else:
        monkeypatch.setenv("MLBLUP_SPARSE_TAIL", mode)
    wl, nu, tree, bas, s = _both(k, n, nu)
    level = tree.max_depth - up
    g = s.loglik_sparse(dev(wl.z), level, tau)
    d = s.loglik(dev(wl.z), level, tau=tau)
    info = s.loglik_sparse_info(level, tau)
    kap = _cond_sparse(wl, nu, tree, bas, level, tau)
    tq = max(1e-12, 50 * kap * 2.2e-16)
    say(f"sparse factor tail={mode} cfg{k} n={n} level={level} tau={tau}: tail rows {info['tail_rows']} of "
        f"{info['rows']}, block columns {info['block_columns']}")
    if mode == "none":
        assert info["tail_rows"] == 0
    if mode == "all":
        assert info["tail_rows"] == info["rows"] and info["block_columns"] == 0
    if mode == "cap128":
        assert info["tail_rows"] <= 128
    assert abs(g["logdet"] - d["logdet"]) < tq * d["rows"]
    assert abs(g["quad"] - d["quad"]) < tq * abs(d["quad"])
