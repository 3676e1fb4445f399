"""Pins of the oracle's operator tables to the numbers the paper prints
(Sec. 2.1): the weights of the biased and central first-derivative operators
and the matrix M of the compact second-derivative operator.  The fixtures
under tests/golden/ are transcribed from the paper, not computed."""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


@pytest.mark.parametrize("row", _rows("operator_weights.txt"), ids=lambda r: r[0])
def test_first_derivative_weights_match_the_printed_stencils(row):
    name, scale, w = row[0], float(row[1]), [float(v) for v in row[2:]]
    dx = 0.37
    for j in range(5):
        e = np.zeros(5)
        e[j] = 1.0
        assert O.op(name, e, dx) * scale * dx == pytest.approx(w[j], abs=1e-14)


def test_compact_second_derivative_matches_the_printed_matrix():
    M = np.array([[float(Fraction(v)) for v in r] for r in _rows("compact_d2_M.txt")])
    assert M.shape == (4, 4)
    B = np.zeros((5, 5))
    B[1:, 1:] += M
    B[:4, :4] -= M
    dx = 2.0  # 4/dx^2 = 1
    for m in range(5):
        for n in range(5):
            k = np.zeros(5)
            z = np.zeros(5)
            k[m] = 1.0
            z[n] = 1.0
            assert O.op_d2(k, z, dx) == pytest.approx(B[m, n], abs=1e-15), (m, n)
