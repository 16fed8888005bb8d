"""Row interchanges composed on the GPU against the sequential swaps they
stand for: the LU's per-panel interchange plans (emu_dgetrf) and the gather
permutation of the triangular solves (emu_dgetrs), on pivot sequences whose
steps keep hitting the same rows, so that the composition follows long
chains (the LAPACK convention of the solvers section: step k swaps rows k
and ipiv[k] - 1, in order)."""
import numpy as np
import pytest
import torch

import matgen
import oracle as O
import paper_2509_23565_amd as emu

pytestmark = pytest.mark.gpu


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _same_bits(a, b):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64))
    return a.shape == b.shape and np.array_equal(a.view(np.int64), b.view(np.int64))


def _sequential_rows(piv, n):
    """Row k of P B is row rows[k] of B: the swaps applied one after another."""
    rows = np.arange(n)
    for k, p1 in enumerate(piv):
        p = int(p1) - 1
        rows[k], rows[p] = rows[p], rows[k]
    return rows


def _clustered_pivots(n, seed):
    """Valid pivots (ipiv[k] - 1 >= k) of which half hit one of five rows at
    the bottom, the rest a near or far row below k or k itself."""
    g = matgen.rng(seed, n)
    hot = n - 1 - np.arange(5)
    piv = np.empty(n, dtype=np.int64)
    for k in range(n):
        u = g.random()
        if u < 0.5:
            p = int(hot[int(g.integers(0, 5))])
        elif u < 0.7:
            p = k + int(g.integers(0, 3))
        elif u < 0.8:
            p = k
        else:
            p = int(g.integers(k, n))
        piv[k] = min(max(p, k), n - 1) + 1
    return piv


@pytest.mark.parametrize("n", [3000, 40000])
def test_solve_permutation_clustered_pivots(n):
    # unit factors (identity): the solve is exactly the row permutation, so
    # the result is B's rows in the order the sequential swaps give; 40000
    # rows take the composition whose row map does not fit in LDS
    piv = _clustered_pivots(n, 5)
    B = matgen.uniform(n, 2, seed=6)
    expect = B[_sequential_rows(piv, n)]
    LU = torch.eye(n, dtype=torch.float64, device="cuda").t()
    Bg = emu.colmajor(B)
    emu.dgetrs(LU, torch.as_tensor(piv.astype(np.int32), device="cuda"), Bg)
    assert _same_bits(_host(Bg), expect)
    del LU
    torch.cuda.empty_cache()


@pytest.mark.parametrize("nb", [64, 256])
def test_getrf_every_pivot_in_the_last_row(nb):
    # rows of an upper triangular U (dominant diagonal) shifted by one: the
    # pivot of every column is the row that the previous step moved to the
    # bottom, so every interchange of every panel targets row n - 1 and the
    # plans compose one chain per panel; factors and pivots bit-exact
    n = 1500
    g = matgen.rng(3, n)
    U = np.triu(g.uniform(-1.0, 1.0, size=(n, n)))
    U[np.diag_indices(n)] = float(n)
    A = np.asfortranarray(U[(np.arange(n) + 1) % n])
    LU, piv, info = O.getrf(A, nb=nb, s=3)
    assert info == 0 and np.all(piv[:-1] == n)
    Ag = emu.colmajor(A)
    ipiv, dinfo = emu.dgetrf(Ag, nb=nb, nslices=3)
    assert int(_host(dinfo)[0]) == 0
    assert np.array_equal(_host(ipiv), piv)
    assert _same_bits(_host(Ag), LU)
