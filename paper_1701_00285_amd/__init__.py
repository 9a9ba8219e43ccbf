"""Multilevel spatial BLUP on AMD MI355X (gfx950).

The solve of the kriging system in a multilevel basis W orthogonal to the
polynomial trend (arXiv:1701.00285, Sec. 5.2): C_W gamma_W = W Z with
C_W = W C W^T, C the dense Matern covariance.  Everything runs in the
native library libmlblup.so (HIP kernels + host C++); this package only
binds it.
"""
from .api import (DLOGRHO, FP32, FP64, MFMA_BF16X3, MFMA_FP32, MIXED_FLEXIBLE, MIXED_RELIABLE, PREC_BLOCK, PREC_COARSE,
                  PREC_JACOBI, VALUE, Basis, PcgOptions, Precond, Solver, Tree, autograd_functions, cov_matvec,
                  cov_matvec_noalloc, cov_workspace_bytes, matern, matern_host, profile_enable, profile_read)
from ._lib import MlblupError

__all__ = ["Tree", "Basis", "Solver", "PcgOptions", "Precond", "PREC_JACOBI", "PREC_BLOCK", "PREC_COARSE", "cov_matvec", "cov_matvec_noalloc", "cov_workspace_bytes", "matern", "matern_host",
           "autograd_functions", "profile_enable", "profile_read", "MlblupError",
           "FP64", "FP32", "MFMA_FP32", "MFMA_BF16X3", "VALUE", "DLOGRHO", "MIXED_FLEXIBLE", "MIXED_RELIABLE"]
