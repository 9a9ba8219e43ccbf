"""ctypes declarations of the C ABI in include/mlblup.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlblup.so")

OK, EINVAL, ERANK, ENOCONV, EBREAKDOWN, EHIP, ESTATE = 0, -1, -2, -3, -4, -5, -6
FP64, FP32, MFMA_FP32, MFMA_BF16X3 = 0, 1, 2, 3
VALUE, DLOGRHO = 1, 2
PREC_JACOBI, PREC_BLOCK, PREC_COARSE = 1, 2, 3
MIXED_FLEXIBLE, MIXED_RELIABLE = 0, 1

_NAMES = {EINVAL: "EINVAL", ERANK: "ERANK", ENOCONV: "ENOCONV", EBREAKDOWN: "EBREAKDOWN", EHIP: "EHIP",
          ESTATE: "ESTATE"}


class Matern(C.Structure):
    _fields_ = [("nu", C.c_double), ("rho", C.c_double), ("sigma2", C.c_double)]


class PcgOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32),
                ("refine_max", C.c_int32), ("history_cap", C.c_int32), ("inner_rtol", C.c_double),
                ("precond", C.c_void_p), ("history_host", C.c_void_p), ("mixed_scheme", C.c_int32),
                ("state_dev", C.c_void_p), ("resume", C.c_int32)]


class PcgInfo(C.Structure):
    _fields_ = [("inner_iters", C.c_int32), ("outer_iters", C.c_int32), ("fp64_matvecs", C.c_int32),
                ("lowp_matvecs", C.c_int32), ("relres_fp64", C.c_double), ("zw_norm", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class MlblupError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I64 = C.c_int64
_I32 = C.c_int32

_SIGS = {
    "mlblup_last_error": (C.c_char_p, []),
    "mlblup_version": (C.c_int32, []),
    "mlblup_build_tree": (C.c_int, [_P, _I64, _I32, _I32, C.POINTER(_P)]),
    "mlblup_tree_info": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32)]),
    "mlblup_tree_perm": (C.c_int, [_P, _P]),
    "mlblup_tree_nodes": (C.c_int, [_P, _P, _P, _P, _P, _P, _P, _P]),
    "mlblup_tree_free": (None, [_P]),
    "mlblup_build_multilevel_basis": (C.c_int, [_P, _I32, C.c_double, C.POINTER(_P)]),
    "mlblup_basis_info": (C.c_int, [_P, C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I64), C.POINTER(_I64)]),
    "mlblup_basis_level_counts": (C.c_int, [_P, _P]),
    "mlblup_basis_transform_bytes": (C.c_int, [_P, _P]),
    "mlblup_matern_host": (C.c_int, [_P, _P, C.c_int64, _P]),
    "mlblup_basis_dense": (C.c_int, [_P, _P, _P]),
    "mlblup_basis_upload": (C.c_int, [_P, _P, _I64, _P]),
    "mlblup_basis_points_dev": (C.c_int, [_P, C.POINTER(_P)]),
    "mlblup_basis_free": (None, [_P]),
    "mlblup_cov_workspace_bytes": (C.c_int, [_I64, _I64, _I32, _I32, _I32, C.POINTER(_I64)]),
    "mlblup_cov_matvec": (C.c_int, [C.POINTER(Matern), _P, _I64, _P, _I64, _I32, _I32, _I32, _P, _P, _P, _P,
                                    _I64, _P]),
    "mlblup_cov_matvec_noalloc": (C.c_int, [C.POINTER(Matern), _P, _I64, _P, _I64, _I32, _I32, _I32, _P, _P, _P,
                                            _P]),
    "mlblup_transform_workspace_bytes": (C.c_int, [_P, C.POINTER(_I64)]),
    "mlblup_apply_W": (C.c_int, [_P, _P, _P, _P, _P, _I64, _P]),
    "mlblup_apply_Wt": (C.c_int, [_P, _P, _P, _P, _P, _I64, _P]),
    "mlblup_solve_workspace_bytes": (C.c_int, [_P, C.POINTER(PcgOpts), _I64, C.POINTER(_I64)]),
    "mlblup_cw_matvec": (C.c_int, [_P, C.POINTER(Matern), _P, _P, _I32, _P, _I64, _P]),
    "mlblup_pcg_solve": (C.c_int, [_P, C.POINTER(Matern), _P, _P, _I32, C.POINTER(PcgOpts), _P, _I64,
                                   C.POINTER(PcgInfo), _P]),
    "mlblup_blup_predict": (C.c_int, [_P, C.POINTER(Matern), _P, _P, _I64, C.POINTER(PcgOpts), _I32, _I32, _P, _P,
                                      _P, _P, _P, _P, _I64, C.POINTER(PcgInfo), _P]),
    "mlblup_blup_grad": (C.c_int, [_P, C.POINTER(Matern), _P, _P, _P, _I32, _P, _P, _P, _I64, _P]),
    "mlblup_dd_workspace_bytes": (C.c_int, [_P, _I64, C.POINTER(_I64)]),
    "mlblup_blup_predict_dd": (C.c_int, [_P, C.POINTER(Matern), _P, _P, _I64, C.c_double, _I32, _P, _P, _P, _P, _P,
                                         _I64, _P]),
    "mlblup_loglik_workspace_bytes": (C.c_int, [_P, _I32, C.POINTER(_I64), C.POINTER(_I64)]),
    "mlblup_loglik": (C.c_int, [_P, C.POINTER(Matern), _P, _I32, C.c_double, _P, _P, _I64, _P]),
    "mlblup_loglik_sparse_workspace_bytes": (C.c_int, [_P, _I32, C.c_double, C.POINTER(_I64), _P]),
    "mlblup_loglik_sparse": (C.c_int, [_P, C.POINTER(Matern), _P, _I32, C.c_double, _P, _P, _I64, _P]),
    "mlblup_mle_rho_sparse": (C.c_int, [_P, C.POINTER(Matern), _P, _I32, C.c_double, C.c_double, C.c_double,
                                        C.c_double, _P, _P, _I64, _P]),
    "mlblup_mle_nu_rho_sparse": (C.c_int, [_P, C.c_double, _P, _I32, C.c_double, C.c_double, C.c_double,
                                           C.c_double, C.c_double, C.c_double, C.c_double, _P, _P, _I64, _P]),
    "mlblup_sparsity_pattern": (C.c_int, [_P, _I32, C.c_double, C.POINTER(_I64), _P]),
    "mlblup_mle_rho": (C.c_int, [_P, C.POINTER(Matern), _P, _I32, C.c_double, C.c_double, C.c_double, C.c_double, _P,
                                 _P, _I64, _P]),
    "mlblup_mle_nu_rho": (C.c_int, [_P, C.c_double, _P, _I32, C.c_double, C.c_double, C.c_double, C.c_double,
                                    C.c_double, C.c_double, C.c_double, _P, _P, _I64, _P]),
    "mlblup_precond_workspace_bytes": (C.c_int, [_P, C.POINTER(_I64)]),
    "mlblup_precond_build": (C.c_int, [_P, C.POINTER(Matern), _I32, _P, _I64, _P, C.POINTER(_P)]),
    "mlblup_precond_info": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64), C.POINTER(_I64)]),
    "mlblup_precond_workspace_bytes_kind": (C.c_int, [_P, _I32, C.POINTER(_I64)]),
    "mlblup_precond_coarse": (C.c_int, [_P, C.POINTER(_I64), C.POINTER(_I64), _P]),
    "mlblup_precond_upload": (C.c_int, [_P, _P, _I64, _P]),
    "mlblup_precond_blocks": (C.c_int, [_P, _P, _P, _P]),
    "mlblup_precond_free": (None, [_P]),
    "mlblup_profile_enable": (C.c_int, [_I32]),
    "mlblup_profile_read": (C.c_int, [_P, _P, _P]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1701_00285_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def declared_symbols():
    return sorted(_SIGS)


def check(status):
    if status != OK:
        raise MlblupError(status, lib().mlblup_last_error().decode())
    return status
