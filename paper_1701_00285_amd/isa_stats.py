"""VALU instructions per evaluated pair in the inner loop of the symmetric
pair kernels, read from the gfx950 assembly of this repository's own
sources.

    python -m paper_1701_00285_amd.isa_stats [--out profiles/valu_per_pair_sym_kernel.txt]

The kernel's inner loop is its largest basic block; each evaluated pair
issues exactly one v_rsq_f64 (FP64 kernel) or one v_sqrt_f32 (FP32 kernel),
so VALU instructions / that count = VALU instructions per pair.  The
instruction-issue ceiling of a kernel is then the VALU lane rate (256 CUs x
4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane-instructions/s) divided by that
number, in evaluated (unordered) pairs per second.  The output records a
hash of the sources so that stale counts are not used.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import re
import subprocess
import tempfile
from collections import Counter

from . import build as B

SOURCES = ["paper_1701_00285_amd/csrc/pair_sym.hip", "paper_1701_00285_amd/csrc/pairmath.h"]
# (d, 2 nu): the workloads' shapes
SHAPES = [(3, 3), (5, 5), (10, 1), (20, 1)]


def source_hash(root: str) -> str:
    h = hashlib.sha256()
    for s in SOURCES:
        with open(os.path.join(root, s), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _assembly() -> list[str]:
    with tempfile.TemporaryDirectory() as td:
        out = os.path.join(td, "sym.s")
        cmd = [B.hipcc()] + [f for f in B.FLAGS if f != "-fPIC"] + [
            "--cuda-device-only", "-S", os.path.join(B.CSRC, "pair_sym.hip"), "-o", out]
        subprocess.run(cmd, check=True, capture_output=True)
        with open(out) as f:
            return f.read().split("\n")


def _largest_block(lines: list[str], prefix: str) -> list[str]:
    """Largest basic block of the kernel whose mangled name starts with prefix
    (the template arguments; the parameter list is not matched)."""
    start = next(i for i, l in enumerate(lines) if l.startswith(prefix) and l.split(";")[0].rstrip().endswith(":"))
    end = start + 1
    while not lines[end].startswith(".Lfunc_end"):
        end += 1
    blocks, cur = [], []
    for l in lines[start:end]:
        if re.match(r"^\.LBB\S+:", l):
            blocks.append(cur)
            cur = []
        elif l.startswith("\t") and not l.strip().startswith((";", ".")):
            cur.append(l.strip().split()[0])
    blocks.append(cur)
    return max(blocks, key=len)


def counts() -> dict:
    lines = _assembly()
    res = {}
    for d, nu2 in SHAPES:
        for kind, marker in (("fp64", "v_rsq_f64"), ("fp32", "v_sqrt_f32")):
            name = "sym_kernel" if kind == "fp64" else "sym_kernel_lp"
            sym = f"_ZN3mlb12_GLOBAL__N_1{len(name)}{name}ILi{d}ELi{nu2}ELi1EEEv"
            blk = Counter(_largest_block(lines, sym))
            pairs = sum(v for k, v in blk.items() if k.startswith(marker))
            valu = sum(v for k, v in blk.items() if k.startswith("v_"))
            res[(kind, d, nu2)] = round(valu / pairs, 3)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(B.ROOT, "profiles", "valu_per_pair_sym_kernel.txt"))
    a = ap.parse_args()
    c = counts()
    lines = ["# VALU instructions per evaluated pair in the inner loop of the symmetric pair kernels",
             "# (largest basic block of the gfx950 assembly; one v_rsq_f64 / v_sqrt_f32 per pair)",
             "# command: python -m paper_1701_00285_amd.isa_stats",
             f"source_sha256 = {source_hash(B.ROOT)}",
             "sources = " + " ".join(SOURCES)]
    for (kind, d, nu2), v in sorted(c.items()):
        lines.append(f"{kind}_d{d}_nu2{nu2} = {v}")
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
