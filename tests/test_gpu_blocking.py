"""GPU parity of the blocking-factor study (the performance section compares
the LU with emulated and with FP64 Schur updates over blocking factors 256
to 2048, and times it without pivoting):

* LU without interchanges ("lu_pivot" 0) against the oracle's
  getrf(pivot=False), bit for bit: single-workgroup leaves of both sizes, a
  multi-workgroup tall leaf, a wide matrix;
* a block of 1280 columns (more interchanges than one laswp call takes,
  applied in two chunks), with and without pivoting, bit for bit;
* the native FP64 update ("lu_update" 1, rocBLAS dgemm): the same pivots
  as the oracle's FP64 LU, and factors that satisfy the componentwise
  backward-error bound of Gaussian elimination, |PA - LU| <= gamma_n |L||U|
  (any summation order of the updates meets it; without pivoting the growth
  makes two orders differ far beyond their rounding, so the factors are not
  compared entry by entry);
* the block-size autotuner: the recorded choice is what nb = 0 selects in
  emu_dgetrf, emu_dgesv_ir and the workspace query, bit for bit, and the
  input is left untouched.
"""
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


def _boosted(m, n, seed):
    # U(-1, 1) with 2 added on the diagonal: no pivot comes near zero, yet
    # partial pivoting still interchanges rows now and then
    A = np.array(matgen.uniform(m, n, seed=seed), order="F")
    d = np.arange(min(m, n))
    A[d, d] += 2.0
    return A


def _getrf(Ag, nb, s, pivot=1, native=0):
    try:
        emu.set_param("lu_pivot", pivot)
        emu.set_param("lu_update", native)
        return emu.dgetrf(Ag, nb=nb, nslices=s)
    finally:
        emu.set_param("lu_pivot", 1)
        emu.set_param("lu_update", 0)


@pytest.mark.parametrize("m,n,nb,s", [(700, 700, 128, 5), (1500, 1500, 256, 7),
                                      (9000, 48, 32, 3), (1000, 1300, 64, 9)])
def test_getrf_without_pivoting_bit_exact(m, n, nb, s):
    A = _boosted(m, n, seed=41)
    Ag = emu.colmajor(A)
    emu.status()
    ipiv, info = _getrf(Ag, nb, s, pivot=0)
    assert emu.status() == 0
    LU, piv, inf = O.getrf(A, nb=nb, s=s, pivot=False)
    assert int(_host(info)[0]) == inf == 0
    assert np.array_equal(_host(ipiv), piv) and np.array_equal(piv, np.arange(1, min(m, n) + 1))
    assert _same_bits(_host(Ag), LU)
    # the pivoted factorization of the same matrix does interchange rows
    ip2, _ = _getrf(emu.colmajor(A), nb, s, pivot=1)
    assert not np.array_equal(_host(ip2), piv)


def test_getrf_without_pivoting_reports_zero_pivot():
    A = _boosted(300, 300, seed=42)
    A[:, 100] = 0.0
    A[100, 100] = 0.0
    Ag = emu.colmajor(A)
    ipiv, info = _getrf(Ag, 64, 5, pivot=0)
    LU, piv, inf = O.getrf(A, nb=64, s=5, pivot=False)
    assert inf == 101 and int(_host(info)[0]) == inf
    got = _host(Ag)
    nan = np.isnan(got) & np.isnan(LU)
    assert bool(np.all(nan | (got.view(np.int64) == LU.view(np.int64))))


@pytest.mark.parametrize("pivot", [1, 0])
def test_getrf_block_of_1280_bit_exact(pivot):
    m = n = 1400
    nb, s = 1280, 3
    A = _boosted(m, n, seed=43) if not pivot else np.array(
        matgen.phi_matrix(m, n, 1.0, seed=43), order="F")
    Ag = emu.colmajor(A)
    ipiv, info = _getrf(Ag, nb, s, pivot=pivot)
    LU, piv, inf = O.getrf(A, nb=nb, s=s, pivot=bool(pivot))
    assert int(_host(info)[0]) == inf
    assert np.array_equal(_host(ipiv), piv)
    assert _same_bits(_host(Ag), LU)


@pytest.mark.parametrize("pivot", [1, 0])
def test_native_update_lu_matches_fp64_oracle(pivot):
    n, nb = 800, 128
    A = _boosted(n, n, seed=44) if not pivot else np.array(
        matgen.uniform(n, n, seed=44), order="F")
    Ag = emu.colmajor(A)
    ipiv, info = _getrf(Ag, nb, 9, pivot=pivot, native=1)
    _, piv, inf = O.getrf(A, nb=nb, s=None, pivot=bool(pivot))
    got = _host(Ag)
    gp = _host(ipiv)
    assert int(_host(info)[0]) == inf == 0
    assert np.array_equal(gp, piv)
    PA = A.copy()
    for c in range(n):
        p = int(gp[c]) - 1
        if p != c:
            PA[[c, p], :] = PA[[p, c], :]
    L = np.tril(got, -1) + np.eye(n)
    U = np.triu(got)
    u = 2.0 ** -53
    gam = n * u / (1 - n * u)
    # the factorization's own error and that of forming L U here: 2 gamma_n
    # |L||U| (Higham, Accuracy and Stability, Thm 9.3 and Sec. 3.5)
    assert np.all(np.abs(PA - L @ U) <= 2 * gam * (np.abs(L) @ np.abs(U)))


def test_getrf_autotune_selects_recorded_block_size():
    n = 1500
    A = matgen.phi_matrix(n, n, 1.0, seed=41)
    Ag = emu.colmajor(A)
    nb, ms = emu.autotune_getrf(Ag, nslices=3, nbs=[128, 256])
    assert nb in (128, 256) and ms > 0.0
    assert _same_bits(_host(Ag), A)                      # the input is untouched
    A0, A1 = emu.colmajor(A), emu.colmajor(A)
    p0, i0 = emu.dgetrf(A0, nb=0, nslices=3)
    p1, i1 = emu.dgetrf(A1, nb=nb, nslices=3)
    LU, piv, _ = O.getrf(A, nb=nb, s=3)
    assert _same_bits(_host(A0), LU) and _same_bits(_host(A1), LU)
    assert np.array_equal(_host(p0), piv) and np.array_equal(_host(p1), piv)
    L = emu.lib()
    assert L.emu_getrf_workspace_bytes(n, n, 0, 3) == L.emu_getrf_workspace_bytes(n, n, nb, 3)
    # the precision form with nb = 0 factors with the recorded block size too
    b = emu.colmajor(matgen.uniform(n, 1, seed=42))
    X0, r0 = emu.dgesv_ir(Ag, b, nb=0, nslices=3)
    X1, r1 = emu.dgesv_ir(Ag, b, nb=nb, nslices=3)
    assert r0["rc"] == 0 and r0["iters"] == r1["iters"]
    assert _same_bits(_host(X0), _host(X1))
