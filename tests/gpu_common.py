"""Shared fixtures for the GPU parity tests."""
import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def dev(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def row_relerr(y, ref, scale):
    """max_i |y_i - ref_i| / scale_i with scale_i = sum_j |phi_ij x_j| (or
    a stand-in magnitude)."""
    return float(np.max(np.abs(y - ref) / np.maximum(scale, 1e-300)))
