"""Address and undefined-behaviour sanitizers over the host C++ of the
library: kd-tree (tree.cpp), multilevel basis (basis.cpp), sparsity pattern
of the estimator (sparsify.cpp), the analysis of its sparse factorization
(sparse_chol.cpp) and the general-nu tables (genu.cpp), built
for the host only with -fsanitize=address,undefined (hipcc --cuda-host-only;
no device code, no GPU) and driven by tests/sanitize_host_driver.cpp over
ordinary, tied, collinear, tiny and 20-dimensional point sets.  The
preconditioner's host driver (precond_host.cpp) interleaves its host
assembly with device copies and kernel launches, so it is exercised by the
GPU tests instead."""
import os
import shutil
import subprocess

import pytest

from conftest import ROOT

CSRC = os.path.join(ROOT, "paper_1701_00285_amd", "csrc")
SOURCES = ["tree.cpp", "basis.cpp", "sparsify.cpp", "genu.cpp"]


def _tool(*cands):
    for c in cands:
        if c and os.path.exists(c):
            return c
    return None


def _build_and_run(tmp_path, sources, driver, ok_line):
    hipcc = _tool("/opt/rocm/bin/hipcc", shutil.which("hipcc"))
    clang = _tool("/opt/rocm/llvm/bin/clang++")
    if not hipcc or not clang:
        pytest.skip("ROCm compiler not available")
    flags = ["-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    for src in sources + [os.path.join(ROOT, "tests", driver)]:
        path = src if os.path.isabs(src) else os.path.join(CSRC, src)
        obj = str(tmp_path / (os.path.basename(path) + ".o"))
        r = subprocess.run([hipcc] + flags + ["-c", path, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    exe = str(tmp_path / "sanitize_driver")
    r = subprocess.run([clang, "-fsanitize=address,undefined", "-o", exe] + objs + ["-lpthread"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-5000:]
    assert ok_line in out, out[-5000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-5000:]
    return out


@pytest.mark.slow
def test_host_code_under_asan_ubsan(tmp_path):
    _build_and_run(tmp_path, SOURCES, "sanitize_host_driver.cpp", "sanitize driver: ok")


@pytest.mark.slow
def test_sparse_factor_analysis_under_asan_ubsan(tmp_path):
    """The host analysis of the sparse block Cholesky (sparse_chol.cpp):
    wavelet vectors orthonormal with vanishing moments, the block structure
    closed under elimination and scheduled by elimination-tree height, and
    the block algorithm of the device kernels, run in plain loops with the
    same indexing, equal to a dense Cholesky of the same sparsified matrix
    (tests/sparse_host_driver.cpp), under the sanitizers."""
    out = _build_and_run(tmp_path, ["tree.cpp", "basis.cpp", "sparsify.cpp", "sparse_chol.cpp"],
                         "sparse_host_driver.cpp", "sparse driver: ok")
    assert "logdet" in out
