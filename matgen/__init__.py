"""Seeded synthetic input generators shared by the tests, the benchmark and the oracle.

This module only builds input matrices; it holds none of the emulation's
arithmetic (no exponent scan, no slicing, no products, no factorization).
Every generator returns a NumPy float64 array in Fortran (column-major) order,
shape (rows, cols), so that ``a.ctypes.data`` with ``lda = rows`` is the
column-major layout the C ABI takes.

Random draws come from NumPy's PCG64 seeded through ``SeedSequence(seed,
spawn_key=(substream,))`` so that A and B of one workload are independent
streams of one seed.  Elements are drawn column by column (column-major draw
order).

Workload families:

* ``uniform``: i.i.d. U(lo, hi) entries; U(-1, 1) is the small plain-method
  workload, U(-1/2, 1/2) is the HPL generator the paper's randomization
  section names as the benign reference input.
* ``phi_matrix``: a = u * exp(phi * g), u ~ U(-1, 1), g ~ N(0, 1), which
  controls the dynamic range of the entries through phi (phi = 0 gives
  U(-1, 1)).  The paper's emulation section explains that a wide range of
  magnitudes inside a row or a column is what costs the split scheme bits.
* ``kappa_matrix``: diagonally scaled matrices of target condition number,
  in two variants (two-sided diagonal scaling of a well-conditioned phi-matrix,
  after the paper's scaling product L_A A R_A; and a randsvd-style product of
  two random Householder reflectors around a geometric spectrum).
* ``turing``, ``wilkinson``, ``dband``: the integer test matrices of the
  paper's parametric-family section (unit lower triangular with -1 below the
  diagonal; the same plus a last column of ones; the variant with only d
  sub-diagonals of -1).
* ``int_matrix``: random integers of a given bit width, for inputs that fit a
  slice count exactly.
* ``parawilk`` / ``parawilk_random``: the paper's three-parameter family
  ParaWilk_n(d, b, alpha) (parametric-family section) and its randomized form
  (randomization section, eqns (15)-(16)).
* ``spd_matrix``: symmetric positive definite matrices for the Cholesky
  variant.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng", "uniform", "phi_matrix", "kappa_matrix", "turing", "wilkinson",
    "dband", "int_matrix", "hpl_uniform", "batched_specs", "parawilk", "parawilk_random",
    "spd_matrix",
]


def rng(seed: int, substream: int = 0) -> np.random.Generator:
    """PCG64 generator for (seed, substream)."""
    ss = np.random.SeedSequence(entropy=int(seed), spawn_key=(int(substream),))
    return np.random.Generator(np.random.PCG64(ss))


def _colmajor(draw_rows_by_col: np.ndarray) -> np.ndarray:
    """(cols, rows) C-order draw -> (rows, cols) Fortran-order matrix (no copy)."""
    return draw_rows_by_col.T


def uniform(rows: int, cols: int, seed: int = 0, substream: int = 0,
            lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    g = rng(seed, substream)
    return _colmajor(g.uniform(lo, hi, size=(cols, rows)))


def hpl_uniform(n: int, seed: int = 0, substream: int = 0) -> np.ndarray:
    """HPL-style U(-1/2, 1/2) square matrix."""
    return uniform(n, n, seed, substream, -0.5, 0.5)


def phi_matrix(rows: int, cols: int, phi: float, seed: int = 0,
               substream: int = 0) -> np.ndarray:
    """a_ij = u_ij * exp(phi * g_ij), u ~ U(-1, 1), g ~ N(0, 1), i.i.d.

    u is drawn for the whole matrix first, then g, both in column-major order.
    """
    g = rng(seed, substream)
    u = g.uniform(-1.0, 1.0, size=(cols, rows))
    if phi != 0.0:
        z = g.standard_normal(size=(cols, rows))
        z *= float(phi)
        np.exp(z, out=z)
        u *= z
        del z
    return _colmajor(u)


def _householder_apply_left(v: np.ndarray, M: np.ndarray) -> np.ndarray:
    # (I - 2 v v^T / v^T v) M
    w = (2.0 / float(v @ v)) * (v @ M)
    M -= np.outer(v, w)
    return M


def kappa_matrix(n: int, phi: float, kappa: float, seed: int = 0,
                 variant: str = "scaled") -> np.ndarray:
    """Square matrix with condition number of order ``kappa``.

    variant="scaled":  A = D_r (G + sigma I) D_c with G a phi-matrix,
        sigma = 2 sqrt(n) rms(G) (so G + sigma I is well conditioned) and
        D_r, D_c log-spaced diagonals, each spanning a factor sqrt(kappa),
        randomly permuted.  Row and column scalings of this kind are absorbed
        by per-row and per-column exponents.
    variant="randsvd": A = H_u diag(sigma) H_v with two random Householder
        reflectors and sigma geometric from 1 down to 1/kappa, formed in O(n^2).
    """
    g = rng(seed, 7)
    if variant == "scaled":
        A = np.array(phi_matrix(n, n, phi, seed, 0), order="F", copy=True)
        sigma = 2.0 * np.sqrt(n) * np.sqrt(np.mean(A * A))
        A[np.diag_indices(n)] += sigma
        half = 0.5 * np.log10(kappa)
        dr = np.logspace(0.0, -half, n)
        dc = np.logspace(0.0, -half, n)
        g.shuffle(dr)
        g.shuffle(dc)
        A *= dr[:, None]
        A *= dc[None, :]
        return A
    if variant == "randsvd":
        sig = np.logspace(0.0, -np.log10(kappa), n)
        u = g.standard_normal(n)
        v = g.standard_normal(n)
        A = np.zeros((n, n), order="F")
        A[np.diag_indices(n)] = sig
        _householder_apply_left(u, A)
        # right reflector: A (I - 2 v v^T / v^T v)
        w = (2.0 / float(v @ v)) * (A @ v)
        A -= np.outer(w, v)
        return np.asfortranarray(A)
    raise ValueError(f"unknown kappa_matrix variant {variant!r}")


def turing(n: int) -> np.ndarray:
    """Unit lower triangular, -1 everywhere below the diagonal."""
    A = -np.tril(np.ones((n, n)), -1)
    A[np.diag_indices(n)] = 1.0
    return np.asfortranarray(A)


def wilkinson(n: int) -> np.ndarray:
    """Turing matrix with its last column set to ones (the classic
    partial-pivoting growth example: unit diagonal, -1 below, ones in the last
    column)."""
    A = turing(n)
    A[:, n - 1] = 1.0
    return A


def dband(n: int, d: int) -> np.ndarray:
    """Unit lower triangular with -1 on the first d sub-diagonals only."""
    A = np.zeros((n, n))
    A[np.diag_indices(n)] = 1.0
    for k in range(1, min(d, n - 1) + 1):
        idx = np.arange(n - k)
        A[idx + k, idx] = -1.0
    return np.asfortranarray(A)


def int_matrix(rows: int, cols: int, bits: int, seed: int = 0,
               substream: int = 0) -> np.ndarray:
    """Random integers with |a| < 2**bits, stored as float64."""
    g = rng(seed, substream)
    hi = (1 << bits) - 1
    v = g.integers(-hi, hi + 1, size=(cols, rows), dtype=np.int64)
    return _colmajor(v.astype(np.float64))


def batched_specs(count: int, seed: int = 0, nmin: int = 64, nmax: int = 1024,
                  phimax: float = 4.0, rhsmax: int = 8):
    """Sizes, phi and right-hand-side counts of a batch of uneven systems:
    n_i ~ U{nmin..nmax}, phi_i ~ U(0, phimax), nrhs_i ~ U{1..rhsmax}; the
    matrix of system i is phi_matrix(n_i, n_i, phi_i, seed, 1000 + i)."""
    g = rng(seed, 999)
    n = g.integers(nmin, nmax + 1, size=count)
    phi = g.uniform(0.0, phimax, size=count)
    nrhs = g.integers(1, rhsmax + 1, size=count)
    return [(int(n[i]), float(phi[i]), int(nrhs[i])) for i in range(count)]


def parawilk(n: int, d: int, b: int, alpha: float) -> np.ndarray:
    """ParaWilk_n(d, b, alpha) of the paper's parametric-family section.

    Unit diagonal; -1 on the first d sub-diagonals (1 <= i - j <= d); the
    value alpha in every entry above the diagonal of each column j (1-based)
    with (j - 1) mod b == 0, j > 1, and of the last column.  The paper defines
    the placement only through its n = 5, d = 5, b = 2 example (columns 3 and
    5 carry the above-diagonal values); this is the reading that reproduces
    it.  d = n - 1, b >= n, alpha = 1 gives the Wilkinson matrix.
    """
    A = dband(n, d)
    cols = [j for j in range(2, n + 1) if (j - 1) % b == 0]
    if n > 1 and n not in cols:
        cols.append(n)
    for j in cols:
        A[: j - 1, j - 1] = alpha
    return np.asfortranarray(A)


def parawilk_random(n: int, d: int, b: int, alpha: float, seed: int = 0,
                    substream: int = 0) -> np.ndarray:
    """Randomized ParaWilk (eqn (16)): 2 u^2 with u ~ U(0, 1) in every entry
    where ParaWilk is zero, the ParaWilk entries kept (the nonzero-pattern
    function of eqn (15) selects the positions; the printed formula writes the
    matrix itself where its pattern is meant).  u is drawn for all n^2
    positions in column-major order."""
    P = parawilk(n, d, b, alpha)
    g = rng(seed, substream)
    u = _colmajor(g.uniform(0.0, 1.0, size=(n, n)))
    R = 2.0 * u * u
    return np.asfortranarray(np.where(P != 0.0, P, R))


def spd_matrix(n: int, phi: float = 0.0, seed: int = 0, substream: int = 0) -> np.ndarray:
    """Symmetric positive definite: A = G G^T / n + I with G a phi-matrix
    (G G^T formed in float64 by the host BLAS; the input is whatever bits it
    produces, shared by every consumer), symmetrized exactly."""
    G = phi_matrix(n, n, phi, seed, substream)
    A = (G @ G.T) / float(n)
    A = np.triu(A) + np.triu(A, 1).T
    A[np.diag_indices(n)] += 1.0
    return np.asfortranarray(A)
