"""Pins of the ParaWilk generator (parametric-family section, eqns (10)-(14)),
its randomization (eqns (15)-(16)) and the scaled-residual harness on the
oracle (Table 1's trend)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import matgen
import oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "parawilk_table1.json")


def _exact_inverse(A):
    """Gauss-Jordan over the rationals (no rounding anywhere)."""
    n = A.shape[0]
    M = [[Fraction(float(A[i, j])) for j in range(n)] + [Fraction(int(i == j)) for j in range(n)]
         for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        piv = M[c][c]
        M[c] = [v / piv for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    return [[M[i][n + j] for j in range(n)] for i in range(n)]


def test_parawilk_n5_d5_b2_is_the_printed_example_and_its_inverse():
    # eqn (14): n = 5, d = 5, b = 2, the above-diagonal values equal to 1
    printed = np.array([[1, 0, 1, 0, 1], [-1, 1, 1, 0, 1], [-1, -1, 1, 0, 1],
                        [-1, -1, -1, 1, 1], [-1, -1, -1, -1, 1]], dtype=float)
    P = matgen.parawilk(5, 5, 2, 1.0)
    assert np.array_equal(P, printed)
    inv = _exact_inverse(P)
    # the printed inverse has +-1/5 where the true inverse has +-1/4 (the
    # printed matrix times the printed inverse is not the identity)
    q = Fraction(1, 4)
    expect = [[Fraction(1, 2), -q, -q, 0, 0], [0, Fraction(1, 2), Fraction(-1, 2), 0, 0],
              [0, 0, Fraction(1, 2), -q, -q], [0, 0, 0, Fraction(1, 2), Fraction(-1, 2)],
              [Fraction(1, 2), q, -q, q, q]]
    assert inv == [[Fraction(v) for v in row] for row in expect]


def test_parawilk_special_cases():
    n = 40
    # full band, no interior alpha columns, alpha = 1: the Wilkinson matrix
    assert np.array_equal(matgen.parawilk(n, n - 1, n, 1.0), matgen.wilkinson(n))
    # alpha = 0: the d-band matrix of eqn (12); its inverse's first column is
    # the generalized Fibonacci sequence (d = 2: Fibonacci)
    P = matgen.parawilk(5, 2, 5, 0.0)
    assert np.array_equal(P, matgen.dband(5, 2))
    inv = _exact_inverse(P)
    assert [inv[i][0] for i in range(5)] == [1, 1, 2, 3, 5]
    # alpha columns: every b-th column after the first, plus the last
    P = matgen.parawilk(12, 3, 4, 0.5)
    upper_cols = [j for j in range(12) if np.any(np.triu(P, 1)[:, j] != 0)]
    assert upper_cols == [4, 8, 11]                  # 0-based: 1-based 5, 9, 12
    assert np.all(np.triu(P, 1)[:4, 4] == 0.5)


def test_randomized_parawilk_keeps_the_pattern_and_fills_the_zeros():
    n = 300
    P = matgen.parawilk(n, 4, 15, 0.5)
    A = matgen.parawilk_random(n, 4, 15, 0.5, seed=3)
    nz = P != 0
    assert np.array_equal(A[nz], P[nz])
    R = A[~nz]
    assert np.all((R >= 0.0) & (R < 2.0))
    # 2 u^2 with u ~ U(0,1): mean 2/3, skewed toward 0 (median 1/2)
    assert abs(R.mean() - 2.0 / 3.0) < 0.01
    assert abs(np.median(R) - 0.5) < 0.01


def test_table1_trend_on_the_oracle():
    """Table 1 (n = 256, d = 4, b = 15, alpha = 1/2): each extra split gains
    about 2^7, the test passes (< 16) from 7 splits, 3 splits are ~10^7; the
    paper's 6-split value (39.1) lies inside the spread over seeds."""
    g = json.load(open(GOLDEN))
    six = []
    for seed, row in g["seeds"].items():
        r = [row[str(s)] for s in range(3, 10)]
        for s in range(3, 7):
            ratio = row[str(s)] / row[str(s + 1)]
            assert 2 ** 5 < ratio < 2 ** 9, (seed, s, ratio)
        assert row["3"] > 1e6
        assert row["5"] > 16 and row["7"] < 16
        assert row["9"] < 10 * row["native"] and row["8"] < 10 * row["native"]
        assert all(a > b for a, b in zip(r[:5], r[1:6]))
        six.append(row["6"])
    assert min(six) < 39.14 < max(six)


def test_golden_values_recompute():
    # one seed, every count: the stored values are the oracle's
    g = json.load(open(GOLDEN))
    A = matgen.parawilk_random(256, 4, 15, 0.5, seed=2)
    b = matgen.hpl_uniform(256, seed=2, substream=1)[:, :1]
    for s in (3, 6, 9, None):
        LU, piv, _ = O.getrf(A, nb=64, s=s)
        x = O.getrs(LU, piv, b)
        key = "native" if s is None else str(s)
        assert O.scaled_residual(A, x, b) == g["seeds"]["2"][key]
