"""Plain CPU oracle for FP64 GEMM emulated with INT8 slices, and for the
blocked, partially pivoted LU that uses it for its Schur-complement update.

TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
CPU-baseline leg import this module.  It shares no code with the GPU library
(paper_2509_23565_amd/): no kernels, headers, tables or helpers, and it never
imports the library.  It is deliberately slow and written to be read against
the paper: NumPy arrays in float64, one library matmul per slice pair, and
loops in the paper's order.

What it computes (paper: section "Emulation of FP64 and INT8 Splitting",
equations (1)-(2); section "Dense Numerical Solvers Using FP64 Emulation",
equations (5)-(9)):

* each operand is split into s slices, AB = sum_{i,j} A_i B_j (eqn 2), and the
  products with i + j > t are dropped (the truncation threshold t of the same
  section).  The paper gives no slicing algorithm; the readings used here:
    - a slice is an INT8 digit holding 7 magnitude bits and the element's
      sign, q in [-127, 127];
    - A is scaled per row and B per column by 2^-e with e the frexp exponent
      of the line's largest magnitude (max |x| in [2^(e-1), 2^e)); an all-zero
      line has e = 0; the range example, eqn (3), is what per-line scaling
      addresses;
    - digits are taken by truncation toward zero, r_0 = x 2^-e,
      q_i = trunc(128 r_{i-1}), r_i = 128 r_{i-1} - q_i (all exact in FP64),
      so x = 2^e (sum_i q_i 128^-i + remainder) with |remainder| < 128^-s;
    - the threshold is t = s + 1 (the triangle i + j <= s + 1, s(s+1)/2
      products); t = 2s keeps all s^2 products;
    - slice products are exact integers D_g = sum_{i+j=g} Q^A_i Q^B_j for
      g = 2..t;
    - recombination in a fixed order: S = 0; for g = t down to 2:
      S = fl(S + D_g 2^(-7g)); X = S 2^(e_p + f_q); then
      C = fma(alpha, X, beta C) (beta = 0: fma(alpha, X, 0), C not read);
    - rows of A / columns of B holding Inf or NaN give NaN in the matching
      rows / columns of C.
* LU (eqn (8) Schur complement, partial pivoting as described after it): a
  right-looking blocked factorization whose panel, row interchanges and
  triangular solve are FP64, and whose trailing update
  A22 <- A22 - L21 U12 is the emulated GEMM (alpha = -1, beta = 1) or, for
  the native reference, an FP64 matmul.
* The scaled residual of eqn (9), with eps = 2^-53.

Exactness of the slice products: every digit is an integer of magnitude
<= 127, so every partial sum of Q^A_i Q^B_j (in any order, with or without
fused multiply-add) is an integer of magnitude <= k 127^2, and the sum over
the pairs of one diagonal is <= s k 127^2.  ``slice_products`` asserts that
this bound is below 2^53, which makes every floating-point operation inside
the float64 matmul exact; the test suite checks it against int64 arithmetic.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _clib

DIGIT_BITS = 7
RADIX = float(1 << DIGIT_BITS)          # 128
DIGIT_MAX = (1 << DIGIT_BITS) - 1       # 127
DBL_MIN = np.finfo(np.float64).tiny     # smallest normal, 2^-1022
EPS = 2.0 ** -53                        # unit roundoff used in eqn (9)


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


# --------------------------------------------------------------------------
# splitting (emulation section, eqns (1)-(3))
# --------------------------------------------------------------------------

def line_exponents(X: np.ndarray, axis: int):
    """Exponent per line: axis=1 -> one per row, axis=0 -> one per column.

    Returns (e, bad): e[l] is the frexp exponent of max |x| over the line (0
    for an all-zero or empty line or a line holding a non-finite value), and
    bad[l] is True for lines with an Inf or NaN.
    """
    X = np.asarray(X, dtype=np.float64)
    nlines = X.shape[0] if axis == 1 else X.shape[1]
    if X.size == 0:
        return np.zeros(nlines, np.int64), np.zeros(nlines, bool)
    bad = ~np.isfinite(X).all(axis=axis)
    with np.errstate(invalid="ignore"):
        mx = np.abs(X).max(axis=axis)
    mx = np.where(bad, 0.0, mx)
    _, e = np.frexp(mx)
    return e.astype(np.int64), bad


def slice_digits(X: np.ndarray, e: np.ndarray, bad: np.ndarray, s: int,
                 axis: int) -> np.ndarray:
    """Digits of X scaled per line (axis as in line_exponents).

    Returns Q of shape (s,) + X.shape holding integers in [-127, 127] with
    X = 2^e * sum_i Q[i-1] 128^-i + (remainder below 128^-s) on good lines.
    """
    X = np.asarray(X, dtype=np.float64)
    shift = (-e)[:, None] if axis == 1 else (-e)[None, :]
    r = np.ldexp(X, shift)                 # exact: power-of-two scaling
    if axis == 1:
        r[bad, :] = 0.0
    else:
        r[:, bad] = 0.0
    Q = np.empty((s,) + X.shape)
    for i in range(s):
        y = r * RADIX                      # exact
        q = np.trunc(y)                    # truncation toward zero
        r = y - q                          # exact: the fractional part of y
        Q[i] = q
    return Q


def slice_products(QA: np.ndarray, QB: np.ndarray, t: int) -> dict:
    """D[g] = sum over i + j = g (1 <= i <= sA, 1 <= j <= sB) of
    QA[i-1] @ QB[j-1], g = 2..t.

    QA has shape (sA, m, k), QB (sB, k, n) (sA = sB = s in the method as the
    paper writes it; fewer slices for one operand are the unequal splits).
    Values are exact integers stored in float64 (see the module docstring
    for the bound that makes it so).
    """
    sa, m, k = QA.shape
    sb = QB.shape[0]
    n = QB.shape[2]
    pairs_max = min(sa, sb, t - 1)
    assert pairs_max * k * DIGIT_MAX * DIGIT_MAX < 2.0 ** 53, "slice sum bound"
    D = {}
    for g in range(2, t + 1):
        acc = np.zeros((m, n))
        for i in range(max(1, g - sb), min(sa, g - 1) + 1):
            j = g - i
            acc += QA[i - 1] @ QB[j - 1]
        D[g] = acc
    return D


def recombine(D: dict, t: int, e: np.ndarray, f: np.ndarray, alpha: float,
              beta: float, C: np.ndarray | None) -> np.ndarray:
    """Fixed-order FP64 recombination, then the alpha/beta step (fma)."""
    m = e.shape[0]
    n = f.shape[0]
    S = np.zeros((m, n))
    for g in range(t, 1, -1):
        S = S + np.ldexp(D[g], -DIGIT_BITS * g)      # D exact, scaling exact
    X = np.ldexp(S, e[:, None] + f[None, :])
    out = np.zeros((m, n), order="F") if beta == 0.0 else \
        np.array(C, dtype=np.float64, order="F", copy=True)
    Xf = np.asfortranarray(X)
    _clib.lib().orc_axpby_fma(out.size, float(alpha), _ptr(Xf), float(beta),
                              _ptr(out))
    return out


def dgemm_emu(A, B, s: int, alpha: float = 1.0, beta: float = 0.0, C=None,
              t: int | None = None, return_parts: bool = False, s_b: int | None = None):
    """alpha * emul(A B) + beta * C with s slices per operand, threshold t.

    Default t = s + 1.  s_b (default s) gives B its own slice count (unequal
    splits, related-work section): pairs (i, j) with i <= s, j <= s_b,
    i + j <= t.  BLAS quick returns: m = 0 or n = 0 gives C unchanged; k = 0
    or alpha = 0 gives beta * C (C not read when beta = 0).
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    m, k = A.shape
    k2, n = B.shape
    assert k == k2, "inner dimensions differ"
    if s < 1:
        raise ValueError("s must be >= 1")
    t = s + 1 if t is None else int(t)
    if not (2 <= t <= 2 * s):
        raise ValueError("t must lie in [2, 2s]")
    if m == 0 or n == 0:
        return np.zeros((m, n), order="F") if C is None else np.array(C, order="F")
    if k == 0 or alpha == 0.0:
        if beta == 0.0:
            return np.zeros((m, n), order="F")
        return np.asfortranarray(beta * np.asarray(C, dtype=np.float64))
    e, bad_r = line_exponents(A, axis=1)
    f, bad_c = line_exponents(B, axis=0)
    QA = slice_digits(A, e, bad_r, s, axis=1)
    QB = slice_digits(B, f, bad_c, s if s_b is None else int(s_b), axis=0)
    D = slice_products(QA, QB, t)
    out = recombine(D, t, e, f, alpha, beta, C)
    out[bad_r, :] = np.nan
    out[:, bad_c] = np.nan
    if return_parts:
        return out, dict(e=e, f=f, QA=QA, QB=QB, D=D, bad_r=bad_r, bad_c=bad_c)
    return out


def dgemm_dd(A, B) -> np.ndarray:
    """Reference product: every entry a Dot2 (double-double) dot product."""
    A = np.asfortranarray(A, dtype=np.float64)
    B = np.asfortranarray(B, dtype=np.float64)
    m, k = A.shape
    n = B.shape[1]
    C = np.zeros((m, n), order="F")
    if m and n:
        _clib.lib().orc_dot2_gemm(m, n, k, _ptr(A), max(1, m), _ptr(B),
                                  max(1, k), _ptr(C), max(1, m))
    return C


def rel_err_fro(Chat, Cref) -> float:
    """Normwise relative error ||Chat - Cref||_F / ||Cref||_F."""
    d = np.linalg.norm(np.asarray(Chat) - np.asarray(Cref))
    r = np.linalg.norm(np.asarray(Cref))
    return float(d / r) if r > 0 else float(d)


# --------------------------------------------------------------------------
# LU with partial pivoting (solvers section, eqns (5)-(8))
# --------------------------------------------------------------------------

def _argmax_abs_first(v: np.ndarray) -> int:
    """First index of the largest |v| (NaN counts as largest, first wins)."""
    a = np.abs(v)
    nan = np.isnan(a)
    if nan.any():
        return int(np.argmax(nan))
    return int(np.argmax(a))           # argmax returns the first maximum


def getf2(P: np.ndarray, ipiv: np.ndarray, row0: int, pivot: bool = True) -> int:
    """Unblocked right-looking LU of the panel P (rows x jb) in place.

    Column by column: pick the pivot (first largest magnitude; the diagonal
    entry itself when pivot is False, the performance section's LU without
    pivoting), swap it into place across the panel, scale the column below
    by the reciprocal of the pivot (by division when |pivot| < DBL_MIN), then
    subtract the rank-1 product from the rest of the panel, one rounded
    multiply and one rounded subtract per entry.  ipiv[row0 + c] receives
    the 1-based global row.  Returns the first zero-pivot position (1-based,
    global) or 0.
    """
    rows, jb = P.shape
    info = 0
    for c in range(min(rows, jb)):
        p = c + _argmax_abs_first(P[c:, c]) if pivot else c
        ipiv[row0 + c] = row0 + p + 1
        if P[p, c] != 0.0:
            if p != c:
                P[[c, p], :] = P[[p, c], :]
            piv = P[c, c]
            if abs(piv) >= DBL_MIN:
                P[c + 1:, c] *= 1.0 / piv
            else:
                P[c + 1:, c] /= piv
        elif info == 0:
            info = row0 + c + 1
        if c + 1 < jb:
            P[c + 1:, c + 1:] -= np.outer(P[c + 1:, c], P[c, c + 1:])
    return info


def trsm_unit_lower(L: np.ndarray, B: np.ndarray) -> None:
    """B <- L^-1 B, L unit lower triangular, by forward substitution: for
    each k in increasing order, B[k+1:] -= L[k+1:, k] B[k] (rounded product,
    rounded subtract)."""
    nb = L.shape[0]
    for k in range(nb - 1):
        B[k + 1:, :] -= np.outer(L[k + 1:, k], B[k, :])


def laswp(A: np.ndarray, ipiv: np.ndarray, k1: int, k2: int) -> None:
    """Apply the interchanges ipiv[k1:k2] (1-based rows) to the rows of A, in order."""
    for c in range(k1, k2):
        p = int(ipiv[c]) - 1
        if p != c:
            A[[c, p], :] = A[[p, c], :]


def getrf(A, nb: int = 64, s: int | None = None, t: int | None = None,
          pivot: bool = True):
    """Blocked right-looking LU with partial pivoting, PA = LU (pivot=False:
    no interchanges, A = LU, ipiv the identity; the performance section's
    simplified LU).

    s=None uses an FP64 matmul for the trailing update (native reference);
    otherwise the update is dgemm_emu(L21, U12, s, alpha=-1, beta=1, C=A22).
    Returns (LU, ipiv, info) with LAPACK getrf conventions.
    """
    LU = np.array(A, dtype=np.float64, order="F", copy=True)
    m, n = LU.shape
    mn = min(m, n)
    ipiv = np.zeros(mn, dtype=np.int64)
    info = 0
    for j0 in range(0, mn, nb):
        jb = min(nb, mn - j0)
        j1 = j0 + jb
        pinfo = getf2(LU[j0:, j0:j1], ipiv, j0, pivot)
        if info == 0 and pinfo:
            info = pinfo
        # row interchanges of this panel, applied left and right of it
        for c in range(j0, j1):
            p = int(ipiv[c]) - 1
            if p != c:
                LU[[c, p], :j0] = LU[[p, c], :j0]
                LU[[c, p], j1:] = LU[[p, c], j1:]
        if j1 < n:
            trsm_unit_lower(LU[j0:j1, j0:j1], LU[j0:j1, j1:])
            if j1 < m:
                L21 = LU[j1:, j0:j1]
                U12 = LU[j0:j1, j1:]
                if s is None:
                    LU[j1:, j1:] -= L21 @ U12
                else:
                    LU[j1:, j1:] = dgemm_emu(L21, U12, s, alpha=-1.0, beta=1.0,
                                             C=LU[j1:, j1:], t=t)
    return LU, ipiv, info


# --------------------------------------------------------------------------
# Cholesky (the symmetric case the paper names as a further application of
# the emulated update, solver section and conclusions)
# --------------------------------------------------------------------------

def potf2(P: np.ndarray, row0: int) -> int:
    """Unblocked right-looking Cholesky of the tall panel P (rows x jb, its
    top jb x jb block on the diagonal) in place, lower triangle: column by
    column, l_cc = sqrt(a_cc) (a_cc not positive or NaN: stop and return the
    1-based global column), the column below is multiplied by 1 / l_cc, then
    every a_ij with c < j <= i inside the panel loses l_ic l_jc (one rounded
    multiply, one rounded subtract).  Entries above the diagonal are not
    touched.  Returns 0 or the failing column."""
    rows, jb = P.shape
    for c in range(min(rows, jb)):
        a = P[c, c]
        if not a > 0.0:
            return row0 + c + 1
        l = np.sqrt(a)
        P[c, c] = l
        r = 1.0 / l
        P[c + 1:, c] *= r
        for j in range(c + 1, jb):
            P[j:, j] -= P[j:, c] * P[j, c]
    return 0


def potrf(A, nb: int = 64, s: int | None = None):
    """Blocked right-looking Cholesky A = L L^T of a symmetric matrix, lower
    triangle (the strictly upper part is neither read nor written).

    Per block column: potf2 on the panel A[j0:, j0:j1] (FP64), then the
    trailing update A22 <- A22 - L21 L21^T of the lower triangle, with the
    emulated GEMM (s slices, threshold s + 1; its product of L21 with L21^T
    is exactly symmetric) or an FP64 matmul (s=None).  Returns (L, info):
    info = 0, or the 1-based column whose pivot was not positive, where the
    factorization stops (columns before it are complete, the rest of the
    array is left as it was at that point).
    """
    L = np.array(A, dtype=np.float64, order="F", copy=True)
    n = L.shape[0]
    assert L.shape == (n, n)
    for j0 in range(0, n, nb):
        j1 = min(n, j0 + nb)
        info = potf2(L[j0:, j0:j1], j0)
        if info:
            return L, info
        if j1 < n:
            L21 = L[j1:, j0:j1]
            if s is None:
                upd = L[j1:, j1:] - L21 @ L21.T
            else:
                upd = dgemm_emu(L21, np.asfortranarray(L21.T), s, alpha=-1.0, beta=1.0,
                                C=L[j1:, j1:])
            low = np.tril(np.ones((n - j1, n - j1), dtype=bool))
            L[j1:, j1:] = np.where(low, upd, L[j1:, j1:])
    return L, 0


def getrs(LU, ipiv, B) -> np.ndarray:
    """Solve A X = B from getrf's factors: interchanges, then forward
    substitution with unit L (column order), then back substitution with U
    (x_k = b_k / u_kk, then b[:k] -= U[:k, k] x_k, k decreasing)."""
    LU = np.asarray(LU, dtype=np.float64)
    X = np.array(B, dtype=np.float64, order="F", copy=True)
    squeeze = X.ndim == 1
    if squeeze:
        X = X[:, None]
    n = LU.shape[0]
    laswp(X, ipiv, 0, n)
    for k in range(n - 1):
        X[k + 1:, :] -= np.outer(LU[k + 1:, k], X[k, :])
    for k in range(n - 1, -1, -1):
        X[k, :] = X[k, :] / LU[k, k]
        if k:
            X[:k, :] -= np.outer(LU[:k, k], X[k, :])
    return X[:, 0] if squeeze else X


def residual_dd(A, X, B) -> np.ndarray:
    """B - A X with every entry a Dot2 (double-double) evaluation."""
    A = np.asfortranarray(A, dtype=np.float64)
    X2 = np.asfortranarray(np.atleast_2d(np.asarray(X, dtype=np.float64).T).T)
    B2 = np.asfortranarray(np.atleast_2d(np.asarray(B, dtype=np.float64).T).T)
    n = A.shape[0]
    nrhs = X2.shape[1]
    R = np.zeros((n, nrhs), order="F")
    _clib.lib().orc_dot2_residual(n, nrhs, _ptr(A), max(1, n), _ptr(X2),
                                  max(1, n), _ptr(B2), max(1, n), _ptr(R),
                                  max(1, n))
    return R


def backward_error(A, X, B, R=None) -> float:
    """eta = ||B - AX||_inf / (||A||_inf ||X||_inf + ||B||_inf), the maximum
    over right-hand sides; the residual is evaluated in double-double."""
    A = np.asarray(A, dtype=np.float64)
    X2 = np.atleast_2d(np.asarray(X, dtype=np.float64).T).T
    B2 = np.atleast_2d(np.asarray(B, dtype=np.float64).T).T
    if R is None:
        R = residual_dd(A, X2, B2)
    na = np.abs(A).sum(axis=1).max()
    eta = 0.0
    for j in range(X2.shape[1]):
        den = na * np.abs(X2[:, j]).max() + np.abs(B2[:, j]).max()
        eta = max(eta, float(np.abs(R[:, j]).max() / den))
    return eta


def scaled_residual(A, X, B) -> float:
    """Eqn (9): ||Ax - b||_inf / ((||A||_inf ||x||_inf + ||b||_inf) n eps)."""
    n = np.asarray(A).shape[0]
    return backward_error(A, X, B) / (n * EPS)


def gesv_ir(A, B, nb: int = 64, s: int = 3, tol: float = 1e-15, maxiter: int = 10,
            force_fail: int = 0, s_max: int = 9):
    """Precision form: emulated LU with s slices, FP64 iterative refinement,
    fallback to more slices (this form is not in the paper; its stopping
    quantity is eqn (9)'s scaled residual without the n eps factor).

    1. LU of A with s slices; X = getrs(B).
    2. Repeat: R = B - A X (FP64); eta = max over columns of
       ||R||_inf / (||A||_inf ||X||_inf + ||B||_inf).  Stop when eta <= tol.
       If eta did not fall below half its previous value, or maxiter
       corrections were applied, or eta is NaN: fall back; else X += getrs(R).
    3. Fallback: s = min(s + 2, s_max) and back to 1; at s_max: give up.
    The first ``force_fail`` convergence checks count as failed (test hook).
    Returns (X, info dict with iters, berr, s_final, info, converged).
    """
    A = np.asarray(A, dtype=np.float64)
    B2 = np.atleast_2d(np.asarray(B, dtype=np.float64).T).T
    normA = np.abs(A).sum(axis=1).max()
    total = 0
    while True:
        LU, ipiv, info = getrf(A, nb=nb, s=s)
        if info > 0:
            return None, dict(iters=total, berr=float("nan"), s_final=s, info=info,
                              converged=False)
        X = getrs(LU, ipiv, B2)
        prev = None
        it = 0
        while True:
            R = B2 - A @ X
            eta = 0.0
            for r in range(B2.shape[1]):
                den = normA * np.abs(X[:, r]).max() + np.abs(B2[:, r]).max()
                e = np.abs(R[:, r]).max() / den if den > 0 else np.abs(R[:, r]).max()
                if not e <= eta:
                    eta = e
            forced = force_fail > 0
            if forced:
                force_fail -= 1
            if not forced and eta <= tol:
                return X, dict(iters=total, berr=float(eta), s_final=s, info=0,
                               converged=True)
            if forced or it >= maxiter or (prev is not None and not eta <= 0.5 * prev) \
                    or eta != eta:
                break
            prev = eta
            X = X + getrs(LU, ipiv, R)
            total += 1
            it += 1
        if s >= s_max:
            return X, dict(iters=total, berr=float(eta), s_final=s, info=0,
                           converged=False)
        s = min(s + 2, s_max)


def pa_minus_lu(A, LU, ipiv) -> float:
    """||PA - L U||_F / ||A||_F with the product L U formed in double-double."""
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    PA = np.array(A, order="F", copy=True)
    laswp(PA, ipiv, 0, len(ipiv))
    L = np.tril(LU, -1)
    L[np.diag_indices(min(L.shape))] = 1.0
    U = np.triu(LU)
    return rel_err_fro(dgemm_dd(L[:, :min(LU.shape)], U[:min(LU.shape), :]), PA) \
        if n else 0.0
