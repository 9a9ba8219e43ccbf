"""The C-ABI library loads without a GPU and exports every function that
include/mlblup.h declares; the Python binding declares the same set."""
import os
import re

from conftest import ROOT
from paper_1701_00285_amd import _lib


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "mlblup.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mlblup_[a-zA-Z0-9_]+)\s*\(", txt)))


def test_library_exports_header_symbols():
    lib = _lib.lib()
    names = _header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert names == _lib.declared_symbols()


def test_version_and_error_string():
    lib = _lib.lib()
    assert lib.mlblup_version() >= 100
    assert isinstance(lib.mlblup_last_error(), bytes)
