"""Total-degree design matrix X.  TEST INFRASTRUCTURE.

Paper, Sec. 2 (problem setup): the columns of X are the monomials
x_1^a_1 ... x_d^a_d with |a| <= w (the total-degree set Q^d_w), so
p(d, w) = binomial(d + w, w).  The paper fixes neither the column order
nor the coordinates; this oracle uses raw coordinates and graded
lexicographic order: by total degree, and within one degree by exponent
tuple in decreasing lexicographic order (1, x1, x2, ..., x1^2, x1 x2, ...).
beta-hat is reported in this order; predictions do not depend on it.

Pins (tests/test_oracle_design.py): the count p(d, w) against the values
the paper prints ((2,8)->45, (3,7)->120, (10,4)->1001, (20,3)->1771,
(25,2)->351, fixture tests/golden/p_dw.txt), the order against an
independent enumeration by multisets of variable indices, and the
column values against direct products.
"""
from __future__ import annotations

import math

import numpy as np


def td_exponents(d: int, w: int) -> list[tuple[int, ...]]:
    out = []
    for deg in range(w + 1):
        level = []

        def rec(prefix, remaining, pos):
            if pos == d - 1:
                level.append(tuple(prefix + [remaining]))
                return
            for e in range(remaining, -1, -1):
                rec(prefix + [e], remaining - e, pos + 1)

        rec([], deg, 0)
        out.extend(level)
    return out


def td_count(d: int, w: int) -> int:
    return math.comb(d + w, w)


def design_matrix(x: np.ndarray, w: int) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    n, d = x.shape
    cols = []
    for a in td_exponents(d, w):
        c = np.ones(n)
        for j, e in enumerate(a):
            for _ in range(e):
                c = c * x[:, j]
        cols.append(c)
    return np.stack(cols, axis=1)
