"""VALU instructions per evaluated pair in the inner loop of the symmetric
pair kernels, read from the gfx950 assembly of this repository's own
sources.

    python -m paper_1701_00285_amd.isa_stats [--out profiles/valu_per_pair_sym_kernel.txt]

The kernel's pair loop is taken from the first to the last basic block that
holds a v_rsq_f64 (FP64 kernel) or v_sqrt_f32 (FP32 kernel), one per
evaluated pair, without the sections a conditional branch skips that hold
none (rarely taken paths); VALU instructions / that count = VALU
instructions per pair on the common path.  The
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


def _loop_common_path(lines: list[str], prefix: str, marker: str) -> list[str]:
    """Instructions of the pair loop of the kernel whose mangled name starts
    with prefix (the template arguments; the parameter list is not matched):
    the lines from the first basic block holding a `marker` instruction (one
    per evaluated pair) to the end of the last such block, without the
    sections a conditional branch skips (`s_cbranch_execz L` up to label L,
    or up to the end of the region when L is the loop head) that hold no
    marker: those are the rarely taken paths (the exact
    recomputation of near pairs in the expanded-form kernels)."""
    start = next(i for i, l in enumerate(lines) if l.startswith(prefix) and l.split(";")[0].rstrip().endswith(":"))
    end = start + 1
    while not lines[end].startswith(".Lfunc_end"):
        end += 1
    body = lines[start:end]
    # basic blocks by label
    blocks, cur = [], []
    for l in body:
        if re.match(r"^\.LBB\S+:", l):
            blocks.append(cur)
            cur = [l]
        else:
            cur.append(l)
    blocks.append(cur)
    has = [any(x.strip().startswith(marker) for x in b) for b in blocks]
    first = has.index(True)
    last = len(has) - 1 - has[::-1].index(True)
    region = [l for b in blocks[first:last + 1] for l in b]
    out, skip_to, held = [], None, []
    for l in region:
        lab = re.match(r"^(\.LBB\S+):", l)
        if skip_to is not None:
            if lab and lab.group(1) == skip_to:
                if any(x.startswith(marker) for x in held):
                    out.extend(held)
                skip_to, held = None, []
            elif l.startswith("\t") and not l.strip().startswith((";", ".")):
                held.append(l.strip().split()[0])
            continue
        if l.startswith("\t") and not l.strip().startswith((";", ".")):
            ins = l.strip().split()
            out.append(ins[0])
            if ins[0] == "s_cbranch_execz":
                skip_to = ins[1]
    # a skip whose target is the loop head (a backward branch) runs to the
    # end of the region
    if any(x.startswith(marker) for x in held):
        out.extend(held)
    return out


def counts() -> dict:
    lines = _assembly()
    res = {}
    for d, nu2 in SHAPES:
        for kind, marker in (("fp64", "v_rsq_f64"), ("fp32", "v_sqrt_f32")):
            name = "sym_kernel" if kind == "fp64" else "sym_kernel_lp"
            sym = f"_ZN3mlb12_GLOBAL__N_1{len(name)}{name}ILi{d}ELi{nu2}ELi1EEEv"
            blk = Counter(_loop_common_path(lines, sym, marker))
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
             "# (pair loop of the gfx950 assembly without its rarely taken branches; one v_rsq_f64 / v_sqrt_f32 per pair)",
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
