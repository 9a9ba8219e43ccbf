"""Python binding of libmlblup (C ABI in include/mlblup.h).

Argument marshalling only: every step of the solve runs in the library's
HIP kernels or its host C++.  PyTorch provides device memory (workspaces,
the basis image, vectors) and the current HIP stream.  There is no CPU
fallback: if the library is not built, the first call raises.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass

import numpy as np

from . import _lib as L
from ._lib import check

FP64, FP32, MFMA_FP32, MFMA_BF16X3 = L.FP64, L.FP32, L.MFMA_FP32, L.MFMA_BF16X3
VALUE, DLOGRHO = L.VALUE, L.DLOGRHO
PREC_JACOBI, PREC_BLOCK, PREC_COARSE = L.PREC_JACOBI, L.PREC_BLOCK, L.PREC_COARSE
MIXED_FLEXIBLE, MIXED_RELIABLE = L.MIXED_FLEXIBLE, L.MIXED_RELIABLE


def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def matern(nu, rho, sigma2=1.0):
    return L.Matern(float(nu), float(rho), float(sigma2))


@dataclass
class PcgOptions:
    rtol: float = 1e-8
    max_iter: int = 1000
    precision: int = FP64
    refine_max: int = 200
    inner_rtol: float = 1e-2
    precond: object = None          # Precond (uploaded) or None for P_W = I
    history: object = None          # numpy float64 array receiving |r_k|/|Z_W| per iteration, or None
    mixed_scheme: int = 0           # MIXED_FLEXIBLE or MIXED_RELIABLE (reduced precisions)
    state: object = None            # FP64: device tensor of 2 (N - p) + 8 doubles receiving the Krylov state
    resume: bool = False            # continue the recurrence in `state` (with x0 = the earlier gamma_W)

    def to_c(self):
        hist = None if self.history is None else self.history.ctypes.data
        cap = 0 if self.history is None else int(self.history.size)
        st = None if self.state is None else self.state.data_ptr()
        return L.PcgOpts(self.rtol, self.max_iter, self.precision, self.refine_max, cap, self.inner_rtol,
                         None if self.precond is None else self.precond.h, hist, self.mixed_scheme, st,
                         1 if self.resume else 0)


class Precond:
    """Preconditioner P_W (diag(C_W), its per-cell blocks, or the cell blocks
    of the finest level with one dense coarse block) for a basis and
    fixed kernel parameters, built on the device and uploaded."""

    def __init__(self, basis, kern, kind=PREC_BLOCK, device="cuda"):
        torch = _torch()
        lib = L.lib()
        self._lib = lib
        wb = C.c_int64()
        check(lib.mlblup_precond_workspace_bytes_kind(basis.h, int(kind), C.byref(wb)))
        work = torch.empty(max(wb.value, 256), dtype=torch.uint8, device=device)
        h = C.c_void_p()
        check(lib.mlblup_precond_build(basis.h, C.byref(kern), int(kind), _ptr(work), work.numel(), _stream(),
                                       C.byref(h)))
        self.h = h
        self.kind = kind
        db, nb, be = C.c_int64(), C.c_int64(), C.c_int64()
        check(lib.mlblup_precond_info(h, C.byref(db), C.byref(nb), C.byref(be)))
        self.n_blocks, self.block_entries = nb.value, be.value
        self.buf = torch.empty(max(db.value, 256), dtype=torch.uint8, device=device)
        check(lib.mlblup_precond_upload(h, _ptr(self.buf), self.buf.numel(), _stream()))
        del work

    def coarse(self):
        """(c0, G^-T of the coarse block as an nc x nc numpy array) of the
        coarse kind; (0, empty) for the others."""
        c0, nc = C.c_int64(), C.c_int64()
        check(self._lib.mlblup_precond_coarse(self.h, C.byref(c0), C.byref(nc), None))
        y = np.empty((nc.value, nc.value))
        if nc.value:
            check(self._lib.mlblup_precond_coarse(self.h, None, None, _np_ptr(y)))
        return c0.value, y

    def blocks(self):
        """(list of B_v as numpy arrays, their first coefficient index)."""
        vals = np.empty(self.block_entries)
        woff = np.empty(self.n_blocks, dtype=np.int64)
        mw = np.empty(self.n_blocks, dtype=np.int32)
        check(self._lib.mlblup_precond_blocks(self.h, _np_ptr(vals), _np_ptr(woff), _np_ptr(mw)))
        out, o = [], 0
        for k in range(self.n_blocks):
            m = int(mw[k])
            out.append(vals[o:o + m * m].reshape(m, m))
            o += m * m
        return out, woff

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.mlblup_precond_free(self.h)
            self.h = None


class Tree:
    """kd-tree over host points (n x d float64)."""

    def __init__(self, points, leaf_max: int):
        pts = np.ascontiguousarray(points, dtype=np.float64)
        if pts.ndim != 2:
            raise ValueError("points must be (n, d)")
        self._lib = L.lib()
        h = C.c_void_p()
        check(self._lib.mlblup_build_tree(_np_ptr(pts), pts.shape[0], pts.shape[1], int(leaf_max), C.byref(h)))
        self.h = h
        n, d, nn, md = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int32()
        check(self._lib.mlblup_tree_info(h, C.byref(n), C.byref(d), C.byref(nn), C.byref(md)))
        self.n, self.d, self.n_nodes, self.max_depth = n.value, d.value, nn.value, md.value
        self.perm = np.empty(self.n, dtype=np.int64)
        check(self._lib.mlblup_tree_perm(h, _np_ptr(self.perm)))

    def nodes(self):
        nn = self.n_nodes
        out = dict(begin=np.empty(nn, np.int64), end=np.empty(nn, np.int64), depth=np.empty(nn, np.int32),
                   axis=np.empty(nn, np.int32), left=np.empty(nn, np.int32), right=np.empty(nn, np.int32),
                   threshold=np.empty(nn, np.float64))
        check(self._lib.mlblup_tree_nodes(self.h, *[_np_ptr(out[k]) for k in
                                                    ("begin", "end", "depth", "axis", "left", "right", "threshold")]))
        return out

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.mlblup_tree_free(self.h)
            self.h = None


class Basis:
    """Multilevel basis built on the host from a Tree; `upload()` copies its
    device image into a torch-owned buffer."""

    def __init__(self, tree: Tree, degree_w: int, rank_rtol: float = 1e-10):
        self._lib = L.lib()
        self.tree = tree
        h = C.c_void_p()
        check(self._lib.mlblup_build_multilevel_basis(tree.h, int(degree_w), float(rank_rtol), C.byref(h)))
        self.h = h
        p, lv, nmp, db = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64()
        check(self._lib.mlblup_basis_info(h, C.byref(p), C.byref(lv), C.byref(nmp), C.byref(db)))
        self.p, self.levels, self.n_minus_p, self.device_bytes = p.value, lv.value, nmp.value, db.value
        self.n = tree.n
        self.d = tree.d
        self.buf = None

    def transform_bytes(self):
        """Algorithmic bytes of one apply_W / apply_Wt (blocks + vectors)."""
        b = C.c_int64()
        check(self._lib.mlblup_basis_transform_bytes(self.h, C.byref(b)))
        return b.value

    def level_counts(self):
        out = np.empty(self.levels, dtype=np.int64)
        check(self._lib.mlblup_basis_level_counts(self.h, _np_ptr(out)))
        return out

    def sparsity_pattern(self, level, tau, mask=False):
        """Kept entries of the sparsified C~^n_W (Sec. 4.1 tree search with
        distance tau), and with mask=True also the N~ x N~ boolean pattern
        (rows in the order of W)."""
        nt = int(self.level_counts()[level:].sum())
        nnz = C.c_int64()
        m = np.zeros((nt, nt), dtype=np.uint8) if mask else None
        check(self._lib.mlblup_sparsity_pattern(self.h, int(level), float(tau), C.byref(nnz),
                                                _np_ptr(m) if mask else None))
        return (nnz.value, m.astype(bool)) if mask else nnz.value

    def dense(self):
        """(W, L) with columns in tree order (small N only)."""
        W = np.empty((self.n_minus_p, self.n))
        Lm = np.empty((self.p, self.n))
        check(self._lib.mlblup_basis_dense(self.h, _np_ptr(W), _np_ptr(Lm)))
        return W, Lm

    def upload(self, device="cuda"):
        torch = _torch()
        self.buf = torch.empty(self.device_bytes, dtype=torch.uint8, device=device)
        check(self._lib.mlblup_basis_upload(self.h, _ptr(self.buf), self.device_bytes, _stream()))
        ptr = C.c_void_p()
        check(self._lib.mlblup_basis_points_dev(self.h, C.byref(ptr)))
        off = ptr.value - self.buf.data_ptr()
        self.points_dev = self.buf[off:off + self.n * self.d * 8].view(torch.float64).view(self.n, self.d)
        tw = C.c_int64()
        check(self._lib.mlblup_transform_workspace_bytes(self.h, C.byref(tw)))
        self.transform_ws = torch.empty(tw.value, dtype=torch.uint8, device=device)
        return self

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.mlblup_basis_free(self.h)
            self.h = None


def cov_workspace_bytes(m, n, d, precision=FP64, outputs=VALUE):
    b = C.c_int64()
    check(L.lib().mlblup_cov_workspace_bytes(int(m), int(n), int(d), int(precision), int(outputs), C.byref(b)))
    return b.value


def matern_host(r, nu, rho, sigma2=1.0):
    """sigma2 phi(r) evaluated on the host by the library (numpy in, numpy out)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    out = np.empty_like(r)
    k = matern(nu, rho, sigma2)
    check(L.lib().mlblup_matern_host(C.byref(k), _np_ptr(r), r.size, _np_ptr(out)))
    return out


def cov_matvec(rows, cols, x, nu, rho, sigma2=1.0, precision=FP64, outputs=VALUE, work=None):
    """y = C(rows, cols) x and/or dy = (rho dC/drho) x on the GPU.  rows (m, d),
    cols (n, d), x (n,) are float64 device tensors."""
    torch = _torch()
    m, d = rows.shape
    n = cols.shape[0]
    need = cov_workspace_bytes(m, n, d, precision, outputs)
    if work is None or work.numel() < need:
        work = torch.empty(max(need, 256), dtype=torch.uint8, device=rows.device)
    y = torch.empty(m, dtype=torch.float64, device=rows.device) if outputs & VALUE else None
    dy = torch.empty(m, dtype=torch.float64, device=rows.device) if outputs & DLOGRHO else None
    k = matern(nu, rho, sigma2)
    check(L.lib().mlblup_cov_matvec(C.byref(k), _ptr(rows), m, _ptr(cols), n, d, int(precision), int(outputs),
                                    _ptr(x), _ptr(y), _ptr(dy), _ptr(work), work.numel(), _stream()))
    return y, dy


NOALLOC_SCRATCH_BYTES = 64 << 20   # MLBLUP_NOALLOC_SCRATCH_BYTES


def cov_matvec_noalloc(rows, cols, x, nu, rho, sigma2=1.0, precision=FP64, outputs=VALUE, y=None, dy=None):
    """cov_matvec on the library's static per-device scratch: the library
    allocates nothing; the caller passes the outputs (float64 device tensors
    of length m, allocated here only when not given)."""
    torch = _torch()
    m, d = rows.shape
    n = cols.shape[0]
    if outputs & VALUE and y is None:
        y = torch.empty(m, dtype=torch.float64, device=rows.device)
    if outputs & DLOGRHO and dy is None:
        dy = torch.empty(m, dtype=torch.float64, device=rows.device)
    k = matern(nu, rho, sigma2)
    check(L.lib().mlblup_cov_matvec_noalloc(C.byref(k), _ptr(rows), m, _ptr(cols), n, d, int(precision),
                                            int(outputs), _ptr(x), _ptr(y if outputs & VALUE else None),
                                            _ptr(dy if outputs & DLOGRHO else None), _stream()))
    return y, dy


class Solver:
    """Tree + basis + device state for one point set and trend degree.

    Vectors exchanged with the methods below are in INPUT order unless the
    name says `_tree`; the permutation is applied here (marshalling)."""

    def __init__(self, points, degree_w: int, leaf_max: int, nu: float, rho: float, sigma2: float = 1.0,
                 device="cuda", max_targets: int = 0, rank_rtol: float = 1e-10):
        torch = _torch()
        self.points = np.ascontiguousarray(points, dtype=np.float64)
        self.tree = Tree(self.points, leaf_max)
        self.basis = Basis(self.tree, degree_w, rank_rtol).upload(device)
        self.device = device
        self.nu, self.rho, self.sigma2 = float(nu), float(rho), float(sigma2)
        self.n, self.d, self.p = self.basis.n, self.basis.d, self.basis.p
        self.perm = torch.as_tensor(self.tree.perm, device=device)
        self.inv_perm = torch.empty_like(self.perm)
        self.inv_perm[self.perm] = torch.arange(self.n, device=device)
        self.max_targets = int(max_targets)
        wb = C.c_int64()
        check(L.lib().mlblup_solve_workspace_bytes(self.basis.h, None, self.max_targets, C.byref(wb)))
        self.ws = torch.empty(wb.value, dtype=torch.uint8, device=device)

    # ---- ordering ----
    def to_tree(self, v):
        return v[self.perm]

    def from_tree(self, v):
        return v[self.inv_perm]

    def kernel(self, rho=None):
        return matern(self.nu, self.rho if rho is None else rho, self.sigma2)

    def precond(self, kind=PREC_BLOCK, rho=None):
        return Precond(self.basis, self.kernel(rho), kind, self.device)

    # ---- operators ----
    def apply_W(self, v_tree):
        torch = _torch()
        vw = torch.empty(self.n - self.p, dtype=torch.float64, device=self.device)
        vl = torch.empty(self.p, dtype=torch.float64, device=self.device)
        b = self.basis
        check(L.lib().mlblup_apply_W(b.h, _ptr(v_tree), _ptr(vw), _ptr(vl), _ptr(b.transform_ws),
                                     b.transform_ws.numel(), _stream()))
        return vw, vl

    def apply_Wt(self, vw, vl=None):
        torch = _torch()
        v = torch.empty(self.n, dtype=torch.float64, device=self.device)
        b = self.basis
        check(L.lib().mlblup_apply_Wt(b.h, _ptr(vw), _ptr(vl), _ptr(v), _ptr(b.transform_ws),
                                      b.transform_ws.numel(), _stream()))
        return v

    def cw_matvec(self, vw, precision=FP64, rho=None, out=None):
        """C_W vw = W C W^T vw (the solve's operator) in the pair kernel's
        arithmetic `precision`; vw and the result hold N - p values."""
        torch = _torch()
        if out is None:
            out = torch.empty(self.n - self.p, dtype=torch.float64, device=self.device)
        check(L.lib().mlblup_cw_matvec(self.basis.h, C.byref(self.kernel(rho)), _ptr(vw), _ptr(out), int(precision),
                                       _ptr(self.ws), self.ws.numel(), _stream()))
        return out

    def cov_matvec_tree(self, x_tree, precision=FP64, outputs=VALUE, rho=None):
        k = self.kernel(rho)
        pts = self.basis.points_dev
        return cov_matvec(pts, pts, x_tree, k.nu, k.rho, k.sigma2, precision, outputs)

    # ---- estimator: multilevel log-likelihood ----
    def loglik_workspace(self, level):
        """(bytes, N~) of the log-likelihood at `level` (levels >= level of W)."""
        b, r = C.c_int64(), C.c_int64()
        check(L.lib().mlblup_loglik_workspace_bytes(self.basis.h, int(level), C.byref(b), C.byref(r)))
        return b.value, r.value

    def _loglik_ws(self, level):
        torch = _torch()
        need, _ = self.loglik_workspace(level)
        ws = getattr(self, "_llws", None)
        if ws is None or ws.numel() < need:
            self._llws = None
            ws = self._llws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return ws

    def loglik(self, z, level, rho=None, nu=None, tau=math.inf):
        """Multilevel log-likelihood of z (input order) at `level`; a finite
        tau sparsifies C^n_W by the kd-tree search (Sec. 4.1):
        dict(loglik, logdet, quad, rows=N~, nnz=kept entries)."""
        k = self.kernel(rho)
        if nu is not None:
            k = matern(nu, k.rho, k.sigma2)
        ws = self._loglik_ws(level)
        out = np.zeros(4)
        zt = self.to_tree(z).contiguous()
        check(L.lib().mlblup_loglik(self.basis.h, C.byref(k), _ptr(zt), int(level), float(tau), _np_ptr(out),
                                    _ptr(ws), ws.numel(), _stream()))
        return dict(loglik=out[0], logdet=out[1], quad=out[2], rows=self.loglik_workspace(level)[1], nnz=int(out[3]))

    def loglik_sparse_info(self, level, tau):
        """Sparse factorization of C~^n_W at (level, tau): dict(bytes, rows=N~,
        kept, factor_entries, block_columns (before the dense tail), heights,
        flops (of those columns), tail_rows, tail_flops)."""
        b = C.c_int64()
        info = np.zeros(8)
        check(L.lib().mlblup_loglik_sparse_workspace_bytes(self.basis.h, int(level), float(tau), C.byref(b),
                                                           _np_ptr(info)))
        return dict(bytes=b.value, rows=int(info[0]), kept=int(info[1]), factor_entries=int(info[2]),
                    block_columns=int(info[3]), heights=int(info[4]), flops=float(info[5]), tail_rows=int(info[6]),
                    tail_flops=float(info[7]))

    def loglik_sparse(self, z, level, tau, rho=None, nu=None):
        """The log-likelihood of loglik() with the sparse block factorization
        of the kept blocks of C~^n_W (no N x N array): dict(loglik, logdet,
        quad, rows=N~, nnz=kept entries)."""
        k = self.kernel(rho)
        if nu is not None:
            k = matern(nu, k.rho, k.sigma2)
        info = self.loglik_sparse_info(level, tau)
        ws = self._sparse_ws(level, tau)
        out = np.zeros(4)
        zt = self.to_tree(z).contiguous()
        check(L.lib().mlblup_loglik_sparse(self.basis.h, C.byref(k), _ptr(zt), int(level), float(tau), _np_ptr(out),
                                           _ptr(ws), ws.numel(), _stream()))
        return dict(loglik=out[0], logdet=out[1], quad=out[2], rows=info["rows"], nnz=int(out[3]))

    def _sparse_ws(self, level, tau):
        torch = _torch()
        need = self.loglik_sparse_info(level, tau)["bytes"]
        ws = getattr(self, "_spws", None)
        if ws is None or ws.numel() < need:
            self._spws = None
            ws = self._spws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return ws

    def mle_rho(self, z, level, rho_lo, rho_hi, log_rho_tol=1e-6, nu=None, tau=math.inf, sparse=False):
        """Maximum-likelihood rho of the level's log-likelihood (golden
        section on log rho): dict(rho, loglik, evals, bracket).  sparse: each
        evaluation by the sparse block factorization (finite tau)."""
        k = matern(self.nu if nu is None else nu, 1.0, self.sigma2)
        ws = self._sparse_ws(level, tau) if sparse else self._loglik_ws(level)
        fn = L.lib().mlblup_mle_rho_sparse if sparse else L.lib().mlblup_mle_rho
        out = np.zeros(4)
        zt = self.to_tree(z).contiguous()
        check(fn(self.basis.h, C.byref(k), _ptr(zt), int(level), float(tau), float(rho_lo), float(rho_hi),
                 float(log_rho_tol), _np_ptr(out), _ptr(ws), ws.numel(), _stream()))
        return dict(rho=out[0], loglik=out[1], evals=int(out[2]), bracket=out[3])

    def mle_nu_rho(self, z, level, nu_lo, nu_hi, rho_lo, rho_hi, nu_tol=1e-3, log_rho_tol=1e-4, tau=math.inf,
                   sparse=False):
        """Maximum-likelihood (nu, rho) of the level's log-likelihood by the
        profile likelihood (golden section over nu, each point the rho MLE):
        dict(nu, rho, loglik, evals, bracket).  sparse: as in mle_rho."""
        ws = self._sparse_ws(level, tau) if sparse else self._loglik_ws(level)
        fn = L.lib().mlblup_mle_nu_rho_sparse if sparse else L.lib().mlblup_mle_nu_rho
        out = np.zeros(5)
        zt = self.to_tree(z).contiguous()
        check(fn(self.basis.h, float(self.sigma2), _ptr(zt), int(level), float(tau), float(nu_lo), float(nu_hi),
                 float(nu_tol), float(rho_lo), float(rho_hi), float(log_rho_tol), _np_ptr(out), _ptr(ws), ws.numel(),
                 _stream()))
        return dict(nu=out[0], rho=out[1], loglik=out[2], evals=int(out[3]), bracket=out[4])

    # ---- solve / predict / grad ----
    def solve(self, zw, opts: PcgOptions | None = None, x0=None, rho=None, allow_noconv=False):
        torch = _torch()
        opts = opts or PcgOptions()
        gw = x0.clone() if x0 is not None else torch.empty(self.n - self.p, dtype=torch.float64, device=self.device)
        info = L.PcgInfo()
        k = self.kernel(rho)
        co = opts.to_c()
        st = L.lib().mlblup_pcg_solve(self.basis.h, C.byref(k), _ptr(zw), _ptr(gw), 1 if x0 is not None else 0,
                                      C.byref(co), _ptr(self.ws), self.ws.numel(), C.byref(info), _stream())
        if not (allow_noconv and st == L.ENOCONV):
            check(st)
        return gw, info.as_dict(), st

    def predict(self, z, targets=None, opts: PcgOptions | None = None, predict_precision=FP64, rho=None,
                allow_noconv=False, gamma_w0=None):
        """z: (N,) device tensor in input order; targets: (m, d) device tensor.
        Returns dict(zhat, beta (numpy, raw monomials, graded lex), gamma (input
        order), gamma_w, interp_res, info, status)."""
        torch = _torch()
        opts = opts or PcgOptions()
        z_tree = self.to_tree(z).contiguous()
        m = 0 if targets is None else targets.shape[0]
        if m > self.max_targets:
            raise ValueError(f"{m} targets > max_targets={self.max_targets} given at construction")
        zhat = torch.empty(m, dtype=torch.float64, device=self.device) if m else None
        gamma = torch.empty(self.n, dtype=torch.float64, device=self.device)
        gw = gamma_w0.clone() if gamma_w0 is not None else torch.empty(self.n - self.p, dtype=torch.float64,
                                                                       device=self.device)
        beta = np.empty(self.p)
        ires = C.c_double()
        info = L.PcgInfo()
        k = self.kernel(rho)
        co = opts.to_c()
        st = L.lib().mlblup_blup_predict(self.basis.h, C.byref(k), _ptr(z_tree),
                                         _ptr(targets.contiguous()) if m else None, m, C.byref(co),
                                         int(predict_precision), 1 if gamma_w0 is not None else 0, _ptr(zhat),
                                         _np_ptr(beta), _ptr(gamma), _ptr(gw),
                                         C.byref(ires), _ptr(self.ws), self.ws.numel(), C.byref(info), _stream())
        if not (allow_noconv and st == L.ENOCONV):
            check(st)
        return dict(zhat=zhat, beta=beta, gamma=self.from_tree(gamma), gamma_tree=gamma, gamma_w=gw,
                    interp_res=ires.value, info=info.as_dict(), status=st)

    def predict_dd(self, z, targets, rtol=1e-8, max_iter=1000, want_cw=False):
        """The multilevel predictor with P C P^T and K P^T formed in
        double-double (small N; mlblup_blup_predict_dd).  z: (N,) device
        tensor in input order; targets: (m, d) device tensor.  Returns
        dict(zhat, beta, cw (rounded C_W or None), iters, breakdown, relres,
        true_relres)."""
        torch = _torch()
        z_tree = self.to_tree(z).contiguous()
        m = targets.shape[0]
        wb = C.c_int64()
        check(L.lib().mlblup_dd_workspace_bytes(self.basis.h, m, C.byref(wb)))
        work = torch.empty(max(wb.value, 256), dtype=torch.uint8, device=self.device)
        zhat = torch.empty(max(m, 1), dtype=torch.float64, device=self.device)
        nw = self.n - self.p
        cw = torch.empty((nw, nw), dtype=torch.float64, device=self.device) if want_cw else None
        beta = np.empty(self.p)
        info = np.zeros(4)
        k = self.kernel()
        check(L.lib().mlblup_blup_predict_dd(self.basis.h, C.byref(k), _ptr(z_tree), _ptr(targets.contiguous()), m,
                                             float(rtol), int(max_iter), _ptr(zhat), _np_ptr(beta), _ptr(cw),
                                             _np_ptr(info), _ptr(work), work.numel(), _stream()))
        return dict(zhat=zhat[:m], beta=beta, cw=cw, iters=int(info[0]), breakdown=bool(info[1]),
                    relres=float(info[2]), true_relres=float(info[3]))

    def quad_grad(self, z_tree, gamma_tree, lambda_tree=None, precision=FP64, rho=None):
        """(Q, dQ/dlog rho) from gamma = W^T gamma_W (tree order)."""
        q, dq = C.c_double(), C.c_double()
        k = self.kernel(rho)
        check(L.lib().mlblup_blup_grad(self.basis.h, C.byref(k), _ptr(z_tree), _ptr(gamma_tree), _ptr(lambda_tree),
                                       int(precision), C.byref(q) if z_tree is not None else None, C.byref(dq),
                                       _ptr(self.ws), self.ws.numel(), _stream()))
        return (q.value if z_tree is not None else None), dq.value


def _make_autograd():
    torch = _torch()

    class BlupSolve(torch.autograd.Function):
        """gamma_W = C_W(rho)^-1 Z_W as a function of (log rho, Z_W).  Backward
        runs one adjoint solve lambda_W = C_W^-1 g and one fused pass of the
        rho-derivative kernel: dL/dlog rho = -(W^T lambda_W)^T (rho dC/drho)(W^T gamma_W),
        dL/dZ_W = lambda_W."""

        @staticmethod
        def forward(ctx, log_rho, zw, solver, opts):
            rho = float(torch.exp(log_rho.detach()).item())
            gw, info, _ = solver.solve(zw.detach(), opts, rho=rho)
            ctx.solver, ctx.opts, ctx.rho = solver, opts, rho
            ctx.save_for_backward(gw)
            return gw

        @staticmethod
        def backward(ctx, g):
            (gw,) = ctx.saved_tensors
            s = ctx.solver
            lam_w, _, _ = s.solve(g.contiguous(), ctx.opts, rho=ctx.rho)
            gam = s.apply_Wt(gw)
            lam = s.apply_Wt(lam_w)
            _, dq = s.quad_grad(None, gam, lam, rho=ctx.rho)
            # dq = -lam^T (rho dC/drho) gam = dL/dlog rho
            grad_lr = torch.tensor(dq, dtype=torch.float64, device=gw.device) if ctx.needs_input_grad[0] else None
            return grad_lr, (lam_w if ctx.needs_input_grad[1] else None), None, None

    class BlupQuadForm(torch.autograd.Function):
        """Q(rho) = Z_W^T C_W(rho)^-1 Z_W (data term of the multilevel
        likelihood) with dQ/dlog rho = -gamma^T (rho dC/drho) gamma: the
        adjoint of Q is gamma itself, so no extra solve is needed."""

        @staticmethod
        def forward(ctx, log_rho, z_tree, solver, opts):
            rho = float(torch.exp(log_rho.detach()).item())
            zw, _ = solver.apply_W(z_tree)
            gw, info, _ = solver.solve(zw, opts, rho=rho)
            gam = solver.apply_Wt(gw)
            q, dq = solver.quad_grad(z_tree, gam, None, rho=rho)
            ctx.dq = dq
            return torch.tensor(q, dtype=torch.float64, device=z_tree.device)

        @staticmethod
        def backward(ctx, g):
            return g * ctx.dq, None, None, None

    return BlupSolve, BlupQuadForm


_AUTOGRAD = None


def autograd_functions():
    global _AUTOGRAD
    if _AUTOGRAD is None:
        _AUTOGRAD = _make_autograd()
    return _AUTOGRAD


def profile_enable(on=True):
    check(L.lib().mlblup_profile_enable(1 if on else 0))


def profile_read():
    """Per (precision, outputs) bucket: {(prec, outputs): (ms, launches, pairs)}."""
    ms = (C.c_double * 16)()
    n = (C.c_int64 * 16)()
    pairs = (C.c_double * 16)()
    check(L.lib().mlblup_profile_read(ms, n, pairs))
    return {(k // 4, k % 4): (ms[k], n[k], pairs[k]) for k in range(16) if n[k]}
