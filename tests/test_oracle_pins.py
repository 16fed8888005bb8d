"""Pins of the CPU oracle against facts it does not compute itself.

Each test checks the oracle against something the paper or the mathematics
fixes: closed forms of the paper's test matrices (eqns (3), (10)-(12)), exact
integer and rational arithmetic, bounds that follow from the digit
definition, and LAPACK's own pivoting on random inputs.  None of them
re-evaluates the oracle's own formula.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg

import matgen
import oracle as O

U = 2.0 ** -53


def _exact_product(A, B):
    """Exact rational A @ B (tiny sizes only)."""
    m, k = A.shape
    n = B.shape[1]
    FA = [[Fraction(float(A[i, l])) for l in range(k)] for i in range(m)]
    FB = [[Fraction(float(B[l, j])) for j in range(n)] for l in range(k)]
    return [[sum(FA[i][l] * FB[l][j] for l in range(k)) for j in range(n)]
            for i in range(m)]


# ---------------------------------------------------------------- splitting

def test_exponent_brackets_line_maximum():
    A = np.array(matgen.phi_matrix(64, 37, 4.0, seed=3), order="F")
    A[5, :] = 0.0                        # zero row
    A[6, :] = 0.0
    A[6, 3] = 1.0                        # max exactly a power of two
    A[7, :] = 5e-320                     # subnormal row
    A[8, :] *= 1e300
    e, bad = O.line_exponents(A, axis=1)
    assert not bad.any()
    mx = np.abs(A).max(axis=1)
    for p in range(A.shape[0]):
        if mx[p] == 0:
            assert e[p] == 0
        else:
            assert 2.0 ** (int(e[p]) - 1) <= mx[p] < 2.0 ** int(e[p]), p
    f, badc = O.line_exponents(A, axis=0)
    mxc = np.abs(A).max(axis=0)
    for q in range(A.shape[1]):
        assert 2.0 ** (int(f[q]) - 1) <= mxc[q] < 2.0 ** int(f[q])
    A[9, 2] = np.inf
    A[10, 4] = np.nan
    _, bad = O.line_exponents(A, axis=1)
    assert set(np.nonzero(bad)[0]) == {9, 10}


@pytest.mark.parametrize("s", [1, 3, 7, 9])
def test_digits_reconstruct_within_truncation_bound(s):
    A = np.array(matgen.phi_matrix(24, 16, 4.0, seed=11), order="F")
    A[3, :] *= 2.0 ** -1070              # subnormal-range row
    e, bad = O.line_exponents(A, axis=1)
    Q = O.slice_digits(A, e, bad, s, axis=1)
    assert np.all(np.abs(Q) <= 127)
    assert np.all(Q == np.trunc(Q))
    # every digit carries the sign of its element
    assert np.all(Q * np.sign(A)[None] >= 0)
    for p in range(A.shape[0]):
        for l in range(A.shape[1]):
            x = Fraction(float(A[p, l]))
            rec = sum(Fraction(int(Q[i, p, l])) / Fraction(128) ** (i + 1)
                      for i in range(s)) * Fraction(2) ** int(e[p])
            err = abs(x - rec)
            # truncation: the remainder is below one unit of the last digit
            assert err < Fraction(2) ** int(e[p]) / Fraction(128) ** s
            # truncation toward zero never overshoots
            assert abs(rec) <= abs(x)


def test_prefix_property_of_truncated_digits():
    A = np.array(matgen.phi_matrix(50, 40, 2.0, seed=5), order="F")
    e, bad = O.line_exponents(A, axis=0)
    Q9 = O.slice_digits(A, e, bad, 9, axis=0)
    for s in range(1, 9):
        Qs = O.slice_digits(A, e, bad, s, axis=0)
        assert np.array_equal(Qs, Q9[:s])


def test_slice_products_equal_int64_products():
    g = matgen.rng(1)
    s, m, k, n = 4, 9, 4096, 7
    QA = g.integers(-127, 128, size=(s, m, k)).astype(np.float64)
    QB = g.integers(-127, 128, size=(s, k, n)).astype(np.float64)
    QA[:, 0, :] = 127.0                  # worst-case magnitudes
    QB[:, :, 0] = 127.0
    QB[:, :, 1] = -127.0
    for t in (s + 1, 2 * s):
        D = O.slice_products(QA, QB, t)
        for gsum in range(2, t + 1):
            ref = np.zeros((m, n), dtype=np.int64)
            for i in range(1, s + 1):
                j = gsum - i
                if 1 <= j <= s:
                    ref += QA[i - 1].astype(np.int64) @ QB[j - 1].astype(np.int64)
            assert np.array_equal(D[gsum].astype(np.int64), ref)
            assert np.array_equal(D[gsum], ref.astype(np.float64))


# ------------------------------------------------------ emulated products

def test_int8_range_integers_exact_with_one_slice():
    A = matgen.int_matrix(40, 70, 7, seed=2, substream=0)
    B = matgen.int_matrix(70, 30, 7, seed=2, substream=1)
    C = O.dgemm_emu(A, B, 1)
    ref = A.astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(C, ref.astype(np.float64))


def test_exactness_needs_all_pairs_up_to_sa_plus_sb():
    # 21-bit A needs 3 digits, 14-bit B needs 2: the product needs pairs with
    # i + j <= 5; threshold t = s + 1 = 4 drops (3, 2), t = 2s = 6 keeps it.
    A = matgen.int_matrix(32, 64, 21, seed=4, substream=0)
    B = matgen.int_matrix(64, 24, 14, seed=4, substream=1)
    ref = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64)
    assert np.array_equal(O.dgemm_emu(A, B, 3, t=6), ref)
    assert np.array_equal(O.dgemm_emu(A, B, 3, t=5), ref)
    assert not np.array_equal(O.dgemm_emu(A, B, 3, t=4), ref)


def test_range_example_eqn3_as_printed_is_exact_per_row():
    # eqn (3): rows 2^53 and 2^-53 times the identity; per-row exponents
    # keep the small row.
    A = np.array([[2.0 ** 53, 2.0 ** 53], [2.0 ** -53, 2.0 ** -53]], order="F")
    I = np.eye(2, order="F")
    for s in (1, 2, 5):
        assert np.array_equal(O.dgemm_emu(A, I, s), A)


def test_range_example_eqn3_transposed_loses_small_entries():
    # Mixing 2^53 and 2^-53 inside one row: the small entry sits 107 bits
    # below the row's exponent, so it survives only with 7 s >= 107.
    A = np.array([[2.0 ** 53, 2.0 ** -53], [2.0 ** 53, 2.0 ** -53]], order="F")
    I = np.eye(2, order="F")
    C15 = O.dgemm_emu(A, I, 15)
    C16 = O.dgemm_emu(A, I, 16)
    assert C15[0, 1] == 0.0 and C15[0, 0] == 2.0 ** 53
    assert np.array_equal(C16, A)


@pytest.mark.parametrize("s,t", [(2, 3), (3, 4), (4, 8), (7, 8), (9, 10)])
def test_emulated_product_within_truncation_and_rounding_bound(s, t):
    A = np.array(matgen.phi_matrix(5, 9, 3.0, seed=21, substream=0), order="F")
    B = np.array(matgen.phi_matrix(9, 4, 3.0, seed=21, substream=1), order="F")
    alpha, beta = -1.5, 0.75
    C0 = np.array(matgen.uniform(5, 4, seed=21, substream=2), order="F")
    C = O.dgemm_emu(A, B, s, alpha=alpha, beta=beta, C=C0, t=t)
    exact = _exact_product(A, B)
    e, _ = O.line_exponents(A, axis=1)
    f, _ = O.line_exponents(B, axis=0)
    k = A.shape[1]
    # per element: |a b - emulated pair sum| <= 2^(e+f) * delta, with delta
    # from (i) pairs i + j > t dropped, (ii) the remainders of both operands
    dropped = sum(Fraction(127 * 127) / Fraction(128) ** (i + j)
                  for i in range(1, s + 1) for j in range(1, s + 1) if i + j > t)
    delta = dropped + 2 / Fraction(128) ** s + 1 / Fraction(128) ** (2 * s)
    for p in range(5):
        for q in range(4):
            scale = Fraction(2) ** (int(e[p]) + int(f[q]))
            trunc = k * delta * scale
            # recombination: t - 1 rounded adds of terms of magnitude
            # <= k * pairs * 127^2 128^-g; then one rounding in the fma
            terms = sum(k * min(gg - 1, s, 2 * s - gg + 1) * Fraction(127 * 127)
                        / Fraction(128) ** gg for gg in range(2, t + 1)) * scale
            rnd = (t - 1) * Fraction(U) * 2 * terms * abs(Fraction(alpha))
            ref = Fraction(alpha) * exact[p][q] + Fraction(beta) * Fraction(float(C0[p, q]))
            bound = abs(Fraction(alpha)) * trunc + rnd + Fraction(U) * abs(ref) * 2
            assert abs(Fraction(float(C[p, q])) - ref) <= bound


def test_quick_returns():
    A = matgen.uniform(3, 0, seed=1)
    B = matgen.uniform(0, 4, seed=1)
    C0 = np.full((3, 4), 2.0, order="F")
    assert np.array_equal(O.dgemm_emu(A, B, 3, alpha=1.0, beta=0.5, C=C0),
                          np.full((3, 4), 1.0))
    A = matgen.uniform(3, 5, seed=1)
    B = matgen.uniform(5, 4, seed=2)
    Cn = np.full((3, 4), np.nan, order="F")
    # beta = 0: C is not read, NaNs in it are ignored
    assert np.array_equal(O.dgemm_emu(A, B, 3, alpha=0.0, beta=0.0, C=Cn),
                          np.zeros((3, 4)))
    assert np.isfinite(O.dgemm_emu(A, B, 3, alpha=1.0, beta=0.0, C=Cn)).all()


def test_nonfinite_lines_propagate_nan():
    A = np.array(matgen.uniform(6, 8, seed=3), order="F")
    B = np.array(matgen.uniform(8, 5, seed=4), order="F")
    A[2, 1] = np.inf
    B[3, 4] = np.nan
    C = O.dgemm_emu(A, B, 5)
    assert np.isnan(C[2, :]).all() and np.isnan(C[:, 4]).all()
    mask = np.ones_like(C, bool)
    mask[2, :] = False
    mask[:, 4] = False
    assert np.isfinite(C[mask]).all()


@pytest.mark.parametrize("phi", [0.0, 1.0, 4.0])
def test_full_slice_count_meets_1e15_normwise(phi):
    A = matgen.phi_matrix(192, 256, phi, seed=0, substream=0)
    B = matgen.phi_matrix(256, 160, phi, seed=0, substream=1)
    ref = O.dgemm_dd(A, B)
    assert O.rel_err_fro(O.dgemm_emu(A, B, 9), ref) <= 1e-15
    # each extra slice buys roughly 7 bits until rounding takes over
    e7 = O.rel_err_fro(O.dgemm_emu(A, B, 7), ref)
    e5 = O.rel_err_fro(O.dgemm_emu(A, B, 5), ref)
    assert e5 > 1e3 * e7


# -------------------------------------------------------- reference GEMM

def test_dd_gemm_is_correctly_rounded_on_tiny_inputs():
    for seed in range(3):
        A = matgen.phi_matrix(7, 12, 6.0, seed=seed, substream=0)
        B = matgen.phi_matrix(12, 5, 6.0, seed=seed, substream=1)
        C = O.dgemm_dd(A, B)
        exact = _exact_product(A, B)
        for i in range(7):
            for j in range(5):
                assert C[i, j] == float(exact[i][j])   # Fraction -> float rounds to nearest


def test_dd_residual_matches_exact_rational():
    A = matgen.phi_matrix(9, 9, 3.0, seed=8, substream=0)
    X = matgen.uniform(9, 2, seed=8, substream=1)
    B = matgen.uniform(9, 2, seed=8, substream=2)
    R = O.residual_dd(A, X, B)
    AX = _exact_product(A, X)
    for i in range(9):
        for j in range(2):
            assert R[i, j] == float(Fraction(float(B[i, j])) - AX[i][j])


# ------------------------------------------------------------------ LU

@pytest.mark.parametrize("s", [None, 1, 3, 7])
def test_turing_matrix_factors_and_inverse_column(s):
    n = 70
    T = matgen.turing(n)
    LU, ipiv, info = O.getrf(T, nb=16, s=s)
    assert info == 0
    assert np.array_equal(ipiv, np.arange(1, n + 1))     # |1| ties |-1|: first wins
    assert np.array_equal(np.tril(LU, -1), np.tril(T, -1))
    assert np.array_equal(np.triu(LU), np.eye(n))
    e1 = np.zeros(n)
    e1[0] = 1.0
    x = O.getrs(LU, ipiv, e1)
    expect = np.array([1.0] + [2.0 ** (i - 1) for i in range(1, n)])   # eqn (11)
    assert np.array_equal(x, expect)


def test_wilkinson_growth_and_blocked_exactness_threshold():
    n, nb = 100, 32
    W = matgen.wilkinson(n)
    LU, ipiv, info = O.getrf(W, nb=nb, s=None)
    assert np.array_equal(ipiv, np.arange(1, n + 1))
    expect_last = 2.0 ** np.arange(n)                    # U(i, n) = 2^(i-1)
    assert np.array_equal(LU[:, n - 1], np.concatenate([expect_last[:n - 1],
                                                        [2.0 ** (n - 1)]]))
    # U12's last column inside one block spans 2^nb: exact with 7 s >= nb - 1
    good = O.getrf(W, nb=nb, s=5)[0]
    bad = O.getrf(W, nb=nb, s=4)[0]
    assert np.array_equal(good, LU)
    assert not np.array_equal(bad, LU)


@pytest.mark.parametrize("d", [2, 3, 5])
def test_dband_inverse_first_column_is_generalized_fibonacci(d):
    n = 60
    M = matgen.dband(n, d)
    LU, ipiv, info = O.getrf(M, nb=8, s=3)
    e1 = np.zeros(n)
    e1[0] = 1.0
    x = O.getrs(LU, ipiv, e1)
    G = [1]
    for i in range(1, n):
        G.append(sum(G[i - j] for j in range(1, d + 1) if i - j >= 0))
    assert np.array_equal(x, np.array(G, dtype=np.float64))   # eqn (12), d = 2: Fibonacci


def test_native_pivots_match_lapack():
    for seed in range(3):
        A = matgen.phi_matrix(150, 150, 1.0, seed=seed)
        LU, ipiv, info = O.getrf(A, nb=32, s=None)
        lu_ref, piv_ref = scipy.linalg.lu_factor(A)
        assert np.array_equal(ipiv, piv_ref + 1)
        assert np.allclose(LU, lu_ref, rtol=1e-9, atol=1e-12)


def test_pa_equals_lu():
    A = matgen.phi_matrix(200, 200, 1.0, seed=9)
    for s in (None, 9):
        LU, ipiv, info = O.getrf(A, nb=32, s=s)
        assert O.pa_minus_lu(A, LU, ipiv) < 2e-16 * 200 ** 0.5 * 4
    LU, ipiv, info = O.getrf(A, nb=32, s=4)
    r4 = O.pa_minus_lu(A, LU, ipiv)
    assert 1e-12 < r4 < 1e-5     # reduced slices leave their GEMM error in PA - LU


def test_singular_matrix_reports_first_zero_pivot():
    A = np.array(matgen.uniform(40, 40, seed=6), order="F")
    A[:, 17] = 0.0
    for s in (None, 5):
        LU, ipiv, info = O.getrf(A, nb=8, s=s)
        assert info == 18
        assert LU[17, 17] == 0.0
        ref = scipy.linalg.lu_factor(A, check_finite=False)
        assert np.array_equal(ipiv[:17], ref[1][:17] + 1)


def test_lu_without_pivoting_closed_form_and_lapack_on_dominant_columns():
    # 2 x 2 with a tiny leading entry: no interchange, L21 = 1/eps, and
    # U22 = 1 - 1/eps exactly as elimination without pivoting defines it
    A = np.array([[2.0 ** -60, 1.0], [1.0, 1.0]], order="F")
    LU, ipiv, info = O.getrf(A, nb=1, s=None, pivot=False)
    assert info == 0 and list(ipiv) == [1, 2]
    assert LU[1, 0] == 2.0 ** 60 and LU[1, 1] == 1.0 - 2.0 ** 60 and LU[0, 1] == 1.0
    LUp, ipivp, _ = O.getrf(A, nb=1, s=None)
    assert list(ipivp) == [2, 2]                         # partial pivoting swaps
    # a zero leading entry: reported as the first zero pivot, no interchange
    Z = np.array([[0.0, 1.0], [1.0, 1.0]], order="F")
    _, ipz, infz = O.getrf(Z, nb=2, s=None, pivot=False)
    assert infz == 1 and list(ipz) == [1, 2]
    # columns whose diagonal dominates: partial pivoting (LAPACK) makes no
    # interchange, so its factors are those of elimination without pivoting
    n = 60
    G = np.array(matgen.uniform(n, n, seed=31), order="F")
    G[np.arange(n), np.arange(n)] = 2.0 * n
    for nb, s in ((8, None), (16, 9), (7, None)):
        LU, ipiv, info = O.getrf(G, nb=nb, s=s, pivot=False)
        ref_lu, ref_piv = scipy.linalg.lu_factor(G, check_finite=False)
        assert info == 0 and np.array_equal(ipiv, np.arange(1, n + 1))
        assert np.array_equal(ref_piv, np.arange(n))
        assert np.abs(LU - ref_lu).max() <= 1e-13 * np.abs(ref_lu).max()
    # and on a general matrix the two orders differ while both reconstruct A
    M = np.array(matgen.uniform(50, 50, seed=32), order="F")
    LUn, _, _ = O.getrf(M, nb=8, s=None, pivot=False)
    L = np.tril(LUn, -1) + np.eye(50)
    assert np.abs(L @ np.triu(LUn) - M).max() <= 1e-9 * np.abs(M).max() * np.abs(LUn).max()


def test_scaled_residual_matches_eqn9():
    A = matgen.uniform(30, 30, seed=1)
    b = matgen.uniform(30, 1, seed=2)
    LU, ipiv, info = O.getrf(A, nb=8, s=None)
    x = O.getrs(LU, ipiv, b)
    AX = _exact_product(A, x)
    r = max(abs(Fraction(float(b[i, 0])) - AX[i][0]) for i in range(30))
    nA = max(sum(abs(Fraction(float(A[i, j]))) for j in range(30)) for i in range(30))
    den = (nA * max(abs(Fraction(float(v))) for v in x[:, 0])
           + max(abs(Fraction(float(v))) for v in b[:, 0])) * 30 * Fraction(U)
    assert abs(O.scaled_residual(A, x, b) - float(r / den)) <= 1e-12 * float(r / den)
    assert O.scaled_residual(A, x, b) < 16.0


# ------------------------------------------------------- precision form

@pytest.mark.parametrize("s", [3, 4, 5])
def test_refinement_reaches_tolerance_in_double_double(s):
    A = matgen.phi_matrix(300, 300, 1.0, seed=17)
    b = matgen.uniform(300, 2, seed=18)
    X, inf = O.gesv_ir(A, b, nb=32, s=s, tol=1e-15)
    assert inf["converged"] and inf["s_final"] == s
    # judged by the independent double-double residual, not the FP64 one
    assert O.backward_error(A, X, b) <= 1e-15
    assert inf["iters"] >= 1


def test_refinement_fallback_on_forced_failure_and_give_up():
    A = matgen.phi_matrix(200, 200, 1.0, seed=19)
    b = matgen.uniform(200, 1, seed=20)
    X, inf = O.gesv_ir(A, b, nb=32, s=3, tol=1e-15, force_fail=1)
    assert inf["converged"] and inf["s_final"] == 5
    X, inf = O.gesv_ir(A, b, nb=32, s=8, tol=1e-15, force_fail=1)
    assert inf["converged"] and inf["s_final"] == 9
    # a failure at the largest slice count gives up
    X, inf = O.gesv_ir(A, b, nb=32, s=8, tol=1e-15, force_fail=2)
    assert not inf["converged"] and inf["s_final"] == 9


# ----------------------------------------------------------------- Cholesky

def test_cholesky_closed_forms_and_first_nonpositive_pivot():
    L, info = O.potrf(np.array([[4.0, 99.0], [2.0, 5.0]], order="F"), nb=1, s=1)
    assert info == 0
    assert L[0, 0] == 2.0 and L[1, 0] == 1.0 and L[1, 1] == 2.0
    assert L[0, 1] == 99.0                     # the upper part is not touched
    for bad, col in ((-1.0, 6), (0.0, 6), (np.nan, 4)):
        A = np.eye(9, order="F")
        A[col - 1, col - 1] = bad
        for nb in (1, 4, 9):
            L, info = O.potrf(A, nb=nb, s=3)
            assert info == col
            assert np.array_equal(L[:, :col - 1], np.eye(9)[:, :col - 1])


@pytest.mark.parametrize("s", [1, 2, 5, None])
def test_cholesky_recovers_integer_factor_exactly(s):
    # A = B B^T with B unit lower triangular, |b_ij| <= 127: every pivot is
    # 1 and every Schur complement an exact integer, and one 7-bit digit
    # holds each entry of L21, so even one slice reproduces B exactly
    n = 40
    g = np.random.default_rng(5)
    B = np.tril(g.integers(-127, 128, size=(n, n)).astype(np.float64), -1) + np.eye(n)
    A = np.asfortranarray(B @ B.T)
    assert np.abs(A).max() < 2.0 ** 52
    for nb in (3, 8, 16):
        L, info = O.potrf(A, nb=nb, s=s)
        assert info == 0
        assert np.array_equal(np.tril(L), B)
        assert np.array_equal(np.triu(L, 1), np.triu(A, 1))


def test_cholesky_against_lapack_and_symmetric_emulated_product():
    n = 200
    A = matgen.spd_matrix(n, phi=1.0, seed=8)
    ref = scipy.linalg.cholesky(A, lower=True, check_finite=False)
    for nb, s in ((32, None), (48, 9), (64, 7)):
        L, info = O.potrf(A, nb=nb, s=s)
        assert info == 0
        err = np.abs(np.tril(L) - ref).max() / np.abs(ref).max()
        assert err < (1e-13 if s in (None, 9) else 1e-10), (nb, s, err)
    # the trailing update's emulated L21 L21^T is exactly symmetric: pair
    # (i, j) of entry (p, q) is pair (j, i) of entry (q, p), and the scale is
    # 2^(e_p + e_q) either way
    X = np.asfortranarray(matgen.phi_matrix(70, 33, 3.0, seed=9))
    for s in (3, 9):
        P = O.dgemm_emu(X, np.asfortranarray(X.T), s)
        assert np.array_equal(P, P.T)


# ----------------------------------------------------------- unequal splits

def test_unequal_splits_reduce_products_without_changing_exact_digits():
    # B holds integers below 2^14 with one entry of 2^14 - 1 per column, so
    # its columns scale by 2^-14 and two 7-bit digits represent it exactly:
    # every digit of B beyond the second is zero, and giving B two slices
    # instead of nine leaves every diagonal sum, hence every bit, unchanged
    # (17 slice products instead of 45)
    g = np.random.default_rng(21)
    B = g.integers(-(2 ** 14) + 1, 2 ** 14, size=(300, 70)).astype(np.float64)
    B[0, :] = 2.0 ** 14 - 1
    B = np.asfortranarray(B)
    A = np.asfortranarray(matgen.phi_matrix(90, 300, 2.0, seed=22))
    full = O.dgemm_emu(A, B, 9)
    for sb in (2, 3, 5):
        assert np.array_equal(O.dgemm_emu(A, B, 9, s_b=sb).view(np.int64), full.view(np.int64))
    # one slice of B is too few: the second digit carries information
    assert not np.array_equal(O.dgemm_emu(A, B, 9, s_b=1), full)
    # s_b = s is the method itself, and the pair count is the triangle cut
    # to s_b columns: sum over i of min(s_b, t - i)
    assert np.array_equal(O.dgemm_emu(A, B, 9, s_b=9), full)
    _, parts = O.dgemm_emu(A, B, 9, s_b=2, return_parts=True)
    assert parts["QB"].shape[0] == 2
    assert sum(min(2, 10 - i) for i in range(1, 10)) == 17


def test_unequal_splits_exact_for_integers_against_int64():
    # 21-bit A (three digits) times 7-bit B (one digit): exact with s = 3,
    # s_b = 1 (pairs (1..3, 1), all under t = 4), as an int64 product says
    g = np.random.default_rng(23)
    A = g.integers(-(2 ** 21) + 1, 2 ** 21, size=(40, 50))
    B = g.integers(-127, 128, size=(50, 30))
    ref = (A @ B).astype(np.float64)
    got = O.dgemm_emu(np.asfortranarray(A.astype(np.float64)),
                      np.asfortranarray(B.astype(np.float64)), 3, s_b=1)
    assert np.array_equal(got, ref)
