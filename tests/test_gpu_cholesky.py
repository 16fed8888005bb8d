"""GPU parity of the Cholesky variant (emu_dpotrf): lower factor, strictly
upper part untouched, against the oracle's potrf bit for bit; the first
non-positive pivot; the native FP64 update (rocBLAS dsyrk) against the
componentwise backward-error bound of the Cholesky factorization."""
import numpy as np
import pytest
import torch

import matgen
import oracle as O
import paper_2509_23565_amd as emu

pytestmark = pytest.mark.gpu


def _same_bits(a, b):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64))
    return a.shape == b.shape and np.array_equal(a.view(np.int64), b.view(np.int64))


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _spd_with_garbage_upper(n, phi, seed):
    A = np.array(matgen.spd_matrix(n, phi=phi, seed=seed), order="F")
    iu = np.triu_indices(n, 1)
    A[iu] = 1e300          # never read: any use would show in the factor
    return A


# leaves of one and of three workgroups, block sizes that are not multiples
# of the 16-column leaf, slice counts from 3 to 12 (the 12-slice GEMM)
@pytest.mark.parametrize("n,nb,s,phi", [(300, 64, 7, 0.0), (1000, 128, 3, 1.0),
                                        (2200, 256, 9, 1.0), (777, 100, 5, 2.0),
                                        (3000, 512, 4, 1.0), (600, 96, 12, 1.0)])
def test_potrf_bit_exact(n, nb, s, phi):
    A = _spd_with_garbage_upper(n, phi, seed=51)
    Ag = emu.colmajor(A)
    emu.status()
    info = emu.dpotrf(Ag, nb=nb, nslices=s)
    assert emu.status() == 0
    L, inf = O.potrf(A, nb=nb, s=s)
    assert inf == 0 and int(_host(info)[0]) == 0
    assert _same_bits(_host(Ag), L)


@pytest.mark.parametrize("bad,col", [(-1.0, 301), (np.nan, 17), (0.0, 130)])
def test_potrf_reports_first_nonpositive_pivot(bad, col):
    n, nb, s = 400, 64, 5
    A = _spd_with_garbage_upper(n, 1.0, seed=52)
    # a diagonal entry that makes the leading minor of order col indefinite
    # once the earlier columns are eliminated
    A[col - 1, col - 1] = bad
    Ag = emu.colmajor(A)
    info = emu.dpotrf(Ag, nb=nb, nslices=s)
    L, inf = O.potrf(A, nb=nb, s=s)
    assert inf == col and int(_host(info)[0]) == col
    got = _host(Ag)
    assert _same_bits(got[:, :col - 1], L[:, :col - 1])


def test_potrf_native_update_backward_error():
    n, nb = 900, 128
    A = np.array(matgen.spd_matrix(n, phi=1.0, seed=53), order="F")
    Ag = emu.colmajor(A)
    try:
        emu.set_param("lu_update", 1)
        info = emu.dpotrf(Ag, nb=nb, nslices=9)
    finally:
        emu.set_param("lu_update", 0)
    assert int(_host(info)[0]) == 0
    L = np.tril(_host(Ag))
    u = 2.0 ** -53
    gam = (n + 1) * u / (1 - (n + 1) * u)
    # |A - L L^T| <= gamma_(n+1) |L||L|^T (Higham, Thm 10.3), plus the
    # rounding of forming L L^T here
    assert np.all(np.abs(A - L @ L.T) <= 2 * gam * (np.abs(L) @ np.abs(L).T))
    # and the emulated factor at nine slices is close to it
    Ae = emu.colmajor(A)
    emu.dpotrf(Ae, nb=nb, nslices=9)
    Le = np.tril(_host(Ae))
    assert np.abs(Le - L).max() <= 1e-12 * np.abs(L).max()
