"""Pins for oracle.design: p(d, w) against the paper's printed values,
column order against an independent enumeration, values by direct products."""
import itertools
import math

import numpy as np

from conftest import golden
from oracle.design import design_matrix, td_count, td_exponents


def test_counts_match_paper():
    for d, w, p in golden("p_dw.txt"):
        assert td_count(d, w) == p
        if p < 5000:
            assert len(td_exponents(d, w)) == p


def test_order_is_graded_lex():
    for d in (1, 2, 3, 5):
        for w in range(4):
            ref = []
            for deg in range(w + 1):
                for combo in itertools.combinations_with_replacement(range(d), deg):
                    e = [0] * d
                    for j in combo:
                        e[j] += 1
                    ref.append(tuple(e))
            assert td_exponents(d, w) == ref


def test_values():
    rng = np.random.default_rng(3)
    x = rng.random((7, 3))
    X = design_matrix(x, 2)
    for col, e in enumerate(td_exponents(3, 2)):
        np.testing.assert_allclose(X[:, col], np.prod(x ** np.array(e), axis=1), rtol=1e-15)
    assert X.shape == (7, math.comb(5, 2))
