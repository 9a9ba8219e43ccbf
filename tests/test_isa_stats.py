"""The VALU-per-pair counter reads the gfx950 assembly of the symmetric
kernels built from this repository (host-side compile, no GPU)."""
import shutil

import pytest


@pytest.mark.skipif(shutil.which("hipcc") is None and not __import__("os").path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_valu_counts_are_sane():
    from paper_1701_00285_amd import isa_stats
    c = isa_stats.counts()
    for (kind, d, nu2), v in c.items():
        assert 5 < v < 200, (kind, d, nu2, v)
    for d, nu2 in isa_stats.SHAPES:
        if d < 8:
            # both take the distance from differences: FP32 needs fewer instructions
            assert c[("fp32", d, nu2)] < c[("fp64", d, nu2)]
        # at least the distance: d subtractions + d multiply-adds below d = 8 (and always in
        # FP32), d multiply-adds of the FP64 expanded form from d = 8 on
        assert c[("fp64", d, nu2)] >= (2 * d if d < 8 else d)
        assert c[("fp32", d, nu2)] >= 2 * d
