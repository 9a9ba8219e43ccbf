"""Writes gaussian_accuracy_reference.txt: the 100-digit classic BLUP of the
accuracy experiment (Sec. 8, "Prediction numerical accuracy under
ill-conditioning"): Gaussian kernel exp(-r^2 / (2 theta^2)), 200 sites
and 200 targets on the unit disk, Z = 1 + sin(alpha x1) sin(alpha x2),
trend of total degree 8 (p = 45), for each (alpha, theta) of the paper's
table.  The paper's reference had 52 digits; these matrices need about
100 (the results at 100 and 150 digits agree to the last FP64 bit).  Calls
only oracle/ (high-precision classic formulae) and synth/
(inputs).  Run from the repository root:

    python tests/golden/make_gaussian_accuracy_reference.py
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle import highprec  # noqa: E402

W = 8
DPS = 100


def main():
    out = ["# 100-digit classic BLUP of the accuracy experiment (Sec. 8): Gaussian kernel, 200 sites and 200",
           "# targets on the unit disk (synth.accuracy_experiment), trend degree 8 (p = 45).  Written by",
           "# tests/golden/make_gaussian_accuracy_reference.py from oracle.highprec.gaussian_blup.",
           "# Per case: 'case alpha theta', 'sites_checksum' (sum of all site and target coordinates),",
           "# 'kappa_lower' ((max/min Cholesky diagonal)^2 <= cond_2(C)), 'beta' (45 values, graded-lex monomials in",
           "# raw coordinates), 'zhat' (200 values at the targets)."]
    for alpha, theta in synth.ACCURACY_CASES:
        pts, tgt, z = synth.accuracy_experiment(alpha)
        _, _, bs, zs, klb = highprec.gaussian_blup(pts, z, tgt, W, theta, dps=DPS)
        out.append(f"case {alpha!r} {theta!r}")
        out.append(f"sites_checksum {float(np.sum(pts) + np.sum(tgt))!r}")
        out.append(f"kappa_lower {klb}")
        out.append("beta " + " ".join(bs))
        out.append("zhat " + " ".join(zs))
        print(f"alpha={alpha} theta={theta} done", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "gaussian_accuracy_reference.txt"), "w") as f:
        f.write("\n".join(out) + "\n")


if __name__ == "__main__":
    main()
