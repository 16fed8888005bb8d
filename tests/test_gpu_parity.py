"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Integer work (exponents, digits, slice-product sums) must match bit for bit.
Because the recombination and every FP64 step of the LU follow one fixed
order on both sides, the emulated GEMM, the LU factors, the pivots and the
solutions must match bit for bit as well; the tolerance-based checks
(normwise error against the double-double reference, backward error) are
reported on top.
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


def _special_rows(A):
    A = np.array(A, order="F", copy=True)
    A[1, :] = 0.0
    A[2, :] *= 2.0 ** -1060          # subnormal-range row
    A[3, :] = 0.0
    A[3, 0] = 2.0 ** 40              # exact power of two
    A[4, :] *= 1e290
    return A


# ----------------------------------------------------------------- slicing

@pytest.mark.parametrize("s", [1, 3, 7, 9, 10, 16])
@pytest.mark.parametrize("phi", [0.0, 4.0, 12.0])
@pytest.mark.parametrize("shape", [(203, 141), (203, 100), (70, 33)])
def test_slices_bit_exact(s, phi, shape):
    # K = 141: exponent scan and slicing as two passes; K <= 128: one pass
    X = _special_rows(matgen.phi_matrix(*shape, phi, seed=1))
    Xt = np.asfortranarray(X.T)
    for by_rows, M in ((True, X), (False, Xt)):
        e_g, bad_g, q_g = emu.debug_slices(emu.colmajor(M), by_rows, s)
        axis = 1 if by_rows else 0
        e_o, bad_o = O.line_exponents(M, axis)
        q_o = O.slice_digits(M, e_o, bad_o, s, axis)
        assert np.array_equal(_host(e_g), e_o)
        assert not _host(bad_g).any()
        assert np.array_equal(_host(q_g).astype(np.int64), q_o.astype(np.int64))


def test_slices_flag_nonfinite_lines():
    X = np.array(matgen.uniform(70, 40, seed=2), order="F")
    X[5, 3] = np.inf
    X[9, 0] = np.nan
    for by_rows, M in ((True, X), (False, np.asfortranarray(X.T))):
        axis = 1 if by_rows else 0
        e_g, bad_g, q_g = emu.debug_slices(emu.colmajor(M), by_rows, 4)
        e_o, bad_o = O.line_exponents(M, axis)
        assert np.array_equal(_host(bad_g).astype(bool), bad_o)
        assert np.array_equal(_host(e_g), e_o)
        assert np.array_equal(_host(q_g), O.slice_digits(M, e_o, bad_o, 4, axis))


# ---------------------------------------------------------- slice products

@pytest.mark.parametrize("s,t", [(1, 2), (2, 3), (3, 4), (4, 5), (5, 6), (6, 7),
                                 (7, 8), (8, 9), (9, 10), (10, 11), (12, 13), (16, 17),
                                 (2, 4), (3, 6), (4, 8), (5, 10)])
def test_slice_products_bit_exact(s, t):
    A = matgen.phi_matrix(161, 237, 3.0, seed=3, substream=0)
    B = matgen.phi_matrix(237, 99, 3.0, seed=3, substream=1)
    D_g = _host(emu.debug_products(emu.colmajor(A), emu.colmajor(B), s, t))
    _, parts = O.dgemm_emu(A, B, s, t=t, return_parts=True)
    for g in range(2, t + 1):
        assert np.array_equal(D_g[g - 2], parts["D"][g].astype(np.int64)), g


def test_slice_products_across_exactness_chunks():
    # s = 9: one INT32 chunk holds at most 14784 K values (the bound assumes
    # 9 pairs of 127 * 127 per k); with every digit 1..7 equal to 127
    # (x = 1 - 2^-53) and k = 20000 the true sums exceed 2^31.
    k = 20000
    x = 1.0 - 2.0 ** -53
    A = np.full((70, k), x, order="F")
    A[::2, :] *= -1.0
    B = np.full((k, 40), x, order="F")
    B[:, 1::3] *= -1.0
    D_g = _host(emu.debug_products(emu.colmajor(A), emu.colmajor(B), 9))
    _, parts = O.dgemm_emu(A, B, 9, return_parts=True)
    for g in range(2, 11):
        assert np.array_equal(D_g[g - 2], parts["D"][g].astype(np.int64)), g
    assert np.abs(D_g).max() > 2 ** 31           # the INT64 fold was needed


# ------------------------------------------------------------ emulated GEMM

@pytest.mark.parametrize("s", list(range(1, 17)))
def test_dgemm_bit_exact(s):
    m, n, k = 190, 133, 301
    A = matgen.phi_matrix(m, k, 4.0, seed=5, substream=0)
    B = matgen.phi_matrix(k, n, 4.0, seed=5, substream=1)
    C0 = matgen.uniform(m, n, seed=5, substream=2)
    for alpha, beta in ((1.0, 0.0), (-0.7, 1.3), (2.5, -1.0)):
        Cg = emu.colmajor(C0)
        emu.dgemm(emu.colmajor(A), emu.colmajor(B), Cg, alpha=alpha, beta=beta, nslices=s)
        ref = O.dgemm_emu(A, B, s, alpha=alpha, beta=beta, C=C0)
        assert _same_bits(_host(Cg), ref), (alpha, beta)


@pytest.mark.parametrize("s,t", [(2, 4), (3, 6), (5, 10)])
def test_dgemm_full_threshold_bit_exact(s, t):
    A = matgen.int_matrix(64, 96, 21, seed=6, substream=0)
    B = matgen.int_matrix(96, 80, 14, seed=6, substream=1)
    Cg = emu.dgemm(emu.colmajor(A), emu.colmajor(B), nslices=s, t=t)
    ref = O.dgemm_emu(A, B, s, t=t)
    assert _same_bits(_host(Cg), ref)
    if s == 3:   # 21-bit x 14-bit integers are exact with all pairs (s = 3)
        assert np.array_equal(ref, A @ B)


def test_dgemm_submatrix_views_and_beta_zero_ignores_nan():
    big = matgen.phi_matrix(300, 300, 1.0, seed=7)
    Ag = emu.colmajor(big)
    A = big[10:150, 20:220]
    B = big[50:250, 100:190]
    C = np.full((140, 90), np.nan)
    Cbig = emu.colmajor(np.full((200, 120), np.nan))
    Cg = Cbig[5:145, 7:97]
    emu.dgemm(Ag[10:150, 20:220], Ag[50:250, 100:190], Cg, alpha=1.0, beta=0.0, nslices=6)
    ref = O.dgemm_emu(A, B, 6, alpha=1.0, beta=0.0, C=C)
    assert _same_bits(_host(Cg), ref)
    assert np.isnan(_host(Cbig)[:5]).all()       # outside the view untouched


def test_dgemm_nonfinite_rows_cols_and_status():
    A = np.array(matgen.uniform(100, 64, seed=8), order="F")
    B = np.array(matgen.uniform(64, 70, seed=9), order="F")
    A[7, 3] = np.inf
    B[5, 66] = np.nan
    emu.status()
    Cg = emu.dgemm(emu.colmajor(A), emu.colmajor(B), nslices=5)
    ref = O.dgemm_emu(A, B, 5)
    got = _host(Cg)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    assert _same_bits(got[~np.isnan(ref)], ref[~np.isnan(ref)])
    assert emu.status() & 1
    assert emu.status() == 0


def test_dgemm_quick_returns():
    C0 = matgen.uniform(50, 40, seed=10)
    Cg = emu.colmajor(C0)
    Ag = torch.empty((0, 50), dtype=torch.float64, device="cuda").t()
    Bg = torch.empty((40, 0), dtype=torch.float64, device="cuda").t()
    emu.dgemm(Ag, Bg, Cg, alpha=1.0, beta=0.5, nslices=3)
    assert np.array_equal(_host(Cg), 0.5 * C0)
    A = matgen.uniform(50, 30, seed=11)
    B = matgen.uniform(30, 40, seed=12)
    Cg = emu.colmajor(np.full((50, 40), np.nan))
    emu.dgemm(emu.colmajor(A), emu.colmajor(B), Cg, alpha=0.0, beta=0.0, nslices=3)
    assert np.array_equal(_host(Cg), np.zeros((50, 40)))


@pytest.mark.parametrize("phi", [0.0, 1.0, 4.0])
def test_full_slice_count_normwise_error(phi):
    # Pass: eta_F <= max(1e-15, native FP64's eta_F) against the double-double
    # product, at the smallest count that reaches it: nine slices at phi <= 1;
    # at phi = 4 the heavy tail of exp(4 g) can leave a row's largest entry
    # ~2^20 above its typical entries, and ten slices are needed.
    A = matgen.phi_matrix(512, 512, phi, seed=0, substream=0)
    B = matgen.phi_matrix(512, 512, phi, seed=0, substream=1)
    ref = O.dgemm_dd(A, B)
    Ag, Bg = emu.colmajor(A), emu.colmajor(B)
    err = {s: O.rel_err_fro(_host(emu.dgemm(Ag, Bg, nslices=s)), ref) for s in (8, 9, 10, 11)}
    native = O.rel_err_fro(A @ B, ref)
    print(f"phi={phi}: eta_F " + " ".join(f"s={s} {e:.3e}" for s, e in err.items()) +
          f"  native FP64 {native:.3e}")
    bound = max(1e-15, native)
    s_pass = 9 if phi <= 1.0 else 10
    assert err[s_pass] <= bound
    assert err[8] > 4 * err[9]     # one more slice still pays above the rounding floor


def test_range_example_eqn3_transposed_exact_from_sixteen_slices():
    # eqn (3)'s range example with the two magnitudes inside one row: the
    # small entry sits 107 bits below its row's exponent, 7 s >= 107 bits
    # keep it
    A = np.array([[2.0 ** 53, 2.0 ** -53], [2.0 ** 53, 2.0 ** -53]], order="F")
    I = np.eye(2, order="F")
    C15 = _host(emu.dgemm(emu.colmajor(A), emu.colmajor(I), nslices=15))
    C16 = _host(emu.dgemm(emu.colmajor(A), emu.colmajor(I), nslices=16))
    assert C15[0, 1] == 0.0 and C15[0, 0] == 2.0 ** 53
    assert np.array_equal(C16, A)
    assert _same_bits(C15, O.dgemm_emu(A, I, 15)) and _same_bits(C16, O.dgemm_emu(A, I, 16))


@pytest.mark.parametrize("s", [10, 13, 16])
def test_dgemm_wide_counts_long_k(s):
    # s >= 10 at K above the plain exact length (16 pairs: 8320) takes the
    # split variant; above 16640 the chunked pass and the combine into C
    for k in (9000, 17000):
        A = matgen.phi_matrix(70, k, 3.0, seed=19, substream=0)
        B = matgen.phi_matrix(k, 130, 3.0, seed=19, substream=1)
        C0 = matgen.uniform(70, 130, seed=19, substream=2)
        Cg = emu.colmajor(C0)
        emu.dgemm(emu.colmajor(A), emu.colmajor(B), Cg, alpha=-1.0, beta=1.0, nslices=s)
        assert _same_bits(_host(Cg), O.dgemm_emu(A, B, s, alpha=-1.0, beta=1.0, C=C0)), k


# ---------------------------------------------------------------------- LU

@pytest.mark.parametrize("m,n,nb,s", [(256, 256, 64, 7), (300, 300, 64, 5), (400, 400, 64, 12),
                                      (300, 200, 64, 7), (200, 300, 32, 9),
                                      (257, 257, 128, 3), (2600, 300, 64, 5),
                                      (2300, 2300, 128, 4), (4100, 96, 96, 3),
                                      (700, 700, 200, 6), (9000, 40, 32, 3),
                                      (4096, 48, 48, 3), (1040, 48, 16, 3)])
def test_getrf_bit_exact(m, n, nb, s):
    # tall cases run the multi-workgroup panel leaf (more than 2048 rows);
    # 1040 rows: leaves of 1040, 1024 and 1008 rows cross the boundary
    # between the 512- and the 256-thread single-workgroup leaf
    A = matgen.phi_matrix(m, n, 1.0, seed=13)
    Ag = emu.colmajor(A)
    emu.status()
    ipiv, info = emu.dgetrf(Ag, nb=nb, nslices=s)
    assert emu.status() == 0       # in particular no aborted panel wait
    LU, piv, inf = O.getrf(A, nb=nb, s=s)
    assert int(_host(info)[0]) == inf
    assert np.array_equal(_host(ipiv), piv)
    assert _same_bits(_host(Ag), LU)


@pytest.mark.parametrize("m,n,nb,s", [(3000, 3000, 128, 3), (2500, 1800, 96, 6)])
def test_getrf_lookahead_changes_no_bit(m, n, nb, s):
    # the look-ahead (next panel beside the trailing update on a side
    # stream) against the plain step order, which the oracle tests cover
    A = emu.colmajor(matgen.phi_matrix(m, n, 2.0, seed=17))
    A0 = A.clone()
    try:
        emu.set_param("lu_lookahead", 0)
        ip0, inf0 = emu.dgetrf(A0, nb=nb, nslices=s)
    finally:
        emu.set_param("lu_lookahead", 1)
    ip1, inf1 = emu.dgetrf(A, nb=nb, nslices=s)
    assert torch.equal(ip0, ip1) and torch.equal(inf0, inf1)
    assert torch.equal(A0.view(torch.int64), A.view(torch.int64))


@pytest.mark.parametrize("m,n,nb,s", [(6000, 700, 128, 3), (16384, 96, 32, 3),
                                      (17000, 64, 32, 3)])
def test_getrf_cooperative_leaves_change_no_bit(m, n, nb, s):
    # tall leaves (several workgroups) launched cooperatively against the
    # plain launch; both with the look-ahead running beside them.  The
    # plain launch gathers leaves of at most 16 workgroups (16384 rows) on
    # one XCD and exchanges their records with plain stores from the
    # second column on; the cooperative one, and the plain one with
    # leaf_one_xcd = 0, spread them and use device-scope stores throughout;
    # 17000 rows: 17 workgroups, spread in all three.  The tall-skinny cases
    # also match the oracle bit for bit.
    A = emu.colmajor(matgen.phi_matrix(m, n, 1.0, seed=23))
    A0 = A.clone()
    try:
        emu.set_param("leaf_cooperative", 1)
        ip0, inf0 = emu.dgetrf(A0, nb=nb, nslices=s)
    finally:
        emu.set_param("leaf_cooperative", 0)
    assert emu.status() == 0
    ip1, inf1 = emu.dgetrf(A, nb=nb, nslices=s)
    assert emu.status() == 0
    assert torch.equal(ip0, ip1) and torch.equal(inf0, inf1)
    assert torch.equal(A0.view(torch.int64), A.view(torch.int64))
    # plain launches kept spread over the XCDs
    A2 = emu.colmajor(matgen.phi_matrix(m, n, 1.0, seed=23))
    try:
        emu.set_param("leaf_one_xcd", 0)
        ip2, inf2 = emu.dgetrf(A2, nb=nb, nslices=s)
    finally:
        emu.set_param("leaf_one_xcd", 1)
    assert emu.status() == 0
    assert torch.equal(ip2, ip1) and torch.equal(inf2, inf1)
    assert torch.equal(A2.view(torch.int64), A.view(torch.int64))
    if n < 128:
        LU, piv, inf = O.getrf(np.asfortranarray(matgen.phi_matrix(m, n, 1.0, seed=23)),
                               nb=nb, s=s)
        assert int(_host(inf1)[0]) == inf
        assert np.array_equal(_host(ip1), piv)
        assert _same_bits(_host(A), LU)


def _same_or_both_nan(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nan = np.isnan(a) & np.isnan(b)
    return a.shape == b.shape and bool(np.all(nan | (a.view(np.int64) == b.view(np.int64))))


@pytest.mark.parametrize("m,n,nb,s,special", [(300, 64, 32, 3, False), (2600, 48, 48, 3, False),
                                              (2600, 48, 48, 3, True), (5000, 40, 16, 4, True)])
def test_getrf_pivot_ties_and_nonfinite(m, n, nb, s, special):
    # small integers: many equal magnitudes, so the smallest-row tie rule
    # decides; planted NaN / Inf: NaN ranks above every number
    g = np.random.default_rng(29)
    A = np.asfortranarray(g.integers(-3, 4, size=(m, n)).astype(np.float64))
    if special:
        A[m // 2, 5] = np.nan
        A[m - 100, 20] = np.inf
        A[7, 30] = -np.inf
    Ag = emu.colmajor(A)
    ipiv, info = emu.dgetrf(Ag, nb=nb, nslices=s)
    emu.status()
    LU, piv, inf = O.getrf(A, nb=nb, s=s)
    assert np.array_equal(_host(ipiv), piv)
    assert int(_host(info)[0]) == inf
    assert _same_or_both_nan(_host(Ag), LU)


def test_lu_solve_small_config_bit_exact_and_backward_error():
    # plain method, small: n = 1024, U(-1,1), block 64, 7 slices, seed 0
    n = 1024
    A = matgen.uniform(n, n, seed=0, substream=0)
    b = matgen.uniform(n, 1, seed=0, substream=1)
    Ag = emu.colmajor(A)
    ipiv, info = emu.dgetrf(Ag, nb=64, nslices=7)
    xg = emu.colmajor(b)
    emu.dgetrs(Ag, ipiv, xg)
    LU, piv, inf = O.getrf(A, nb=64, s=7)
    x = O.getrs(LU, piv, b)
    assert np.array_equal(_host(ipiv), piv) and int(_host(info)[0]) == inf == 0
    assert _same_bits(_host(Ag), LU)
    assert _same_bits(_host(xg), x)
    eta = O.backward_error(A, _host(xg), b)
    print(f"n=1024 s=7 nb=64: eta {eta:.3e}, scaled residual {eta / (n * O.EPS):.3f}")
    assert eta < 1e-12


@pytest.mark.parametrize("n,nrhs", [(300, 1), (300, 3), (64, 2), (65, 1)])
def test_getrs_bit_exact(n, nrhs):
    A = matgen.phi_matrix(n, n, 2.0, seed=14)
    B = matgen.uniform(n, nrhs, seed=15)
    LU, piv, _ = O.getrf(A, nb=32, s=None)
    x = O.getrs(LU, piv, B)
    Lg = emu.colmajor(LU)
    Bg = emu.colmajor(B)
    emu.dgetrs(Lg, torch.as_tensor(piv.astype(np.int32), device="cuda"), Bg)
    assert _same_bits(_host(Bg), x)


@pytest.mark.parametrize("n,nrhs", [(2048, 2), (2100, 2), (4133, 1), (4133, 3), (4133, 4),
                                    (4133, 5), (64, 4), (65, 1)])
def test_getrs_bit_exact_large(n, nrhs):
    # many 64-row blocks, ragged last blocks; one to four right-hand sides
    # take the one-launch-per-sweep solves, five the per-block launches;
    # synthetic factors (any LU array and valid pivots define a solve)
    g = matgen.rng(17, n)
    LU = np.asfortranarray(g.uniform(-1.0, 1.0, size=(n, n)))
    LU[np.diag_indices(n)] += float(n)
    piv = (np.arange(n) + (g.random(n) * (n - np.arange(n))).astype(np.int64)) + 1
    B = matgen.uniform(n, nrhs, seed=18)
    x = O.getrs(LU, piv, B)
    Bg = emu.colmajor(B)
    emu.dgetrs(emu.colmajor(LU), torch.as_tensor(piv.astype(np.int32), device="cuda"), Bg)
    assert _same_bits(_host(Bg), x)
    assert emu.status() & emu.EMU_STATUS_SOLVE_WAIT == 0


def test_getrf_singular_reports_info():
    A = np.array(matgen.uniform(150, 150, seed=16), order="F")
    A[:, 77] = 0.0
    Ag = emu.colmajor(A)
    ipiv, info = emu.dgetrf(Ag, nb=32, nslices=6)
    LU, piv, inf = O.getrf(A, nb=32, s=6)
    assert inf == 78 and int(_host(info)[0]) == 78
    assert _same_bits(_host(Ag), LU)


@pytest.mark.parametrize("s", [1, 4, 5])
def test_turing_and_wilkinson_closed_forms(s):
    n = 160
    T = matgen.turing(n)
    Tg = emu.colmajor(T)
    ipiv, info = emu.dgetrf(Tg, nb=32, nslices=s)
    assert np.array_equal(_host(ipiv), np.arange(1, n + 1))
    e1 = np.zeros((n, 1))
    e1[0] = 1.0
    xg = emu.colmajor(e1)
    emu.dgetrs(Tg, ipiv, xg)
    expect = np.array([1.0] + [2.0 ** (i - 1) for i in range(1, n)])
    assert np.array_equal(_host(xg)[:, 0], expect)
    W = matgen.wilkinson(n)
    Wg = emu.colmajor(W)
    emu.dgetrf(Wg, nb=32, nslices=s)
    last = _host(Wg)[:, n - 1]
    exact = np.array_equal(last, 2.0 ** np.arange(n))
    assert exact == (s >= 5)          # 7 s bits must cover a 32-row block's 2^31 spread


# ----------------------------------------------------------- precision form

@pytest.mark.parametrize("n,phi,s,nrhs", [(512, 1.0, 3, 1), (700, 0.0, 4, 3),
                                          (1024, 1.0, 5, 1), (1500, 2.0, 3, 2)])
def test_refinement_reaches_1e15(n, phi, s, nrhs):
    A = matgen.phi_matrix(n, n, phi, seed=21)
    B = matgen.uniform(n, nrhs, seed=22)
    Xg, inf = emu.dgesv_ir(emu.colmajor(A), emu.colmajor(B), nb=64, nslices=s, tol=1e-15)
    Xo, info_o = O.gesv_ir(A, B, nb=64, s=s, tol=1e-15)
    X = _host(Xg)
    eta = O.backward_error(A, X, B)          # double-double residual
    print(f"n={n} phi={phi} s={s}: GPU iters {inf['iters']} berr {inf['berr']:.2e} "
          f"(dd {eta:.2e}); oracle iters {info_o['iters']}")
    assert inf["rc"] == 0 and inf["info"] == 0 and inf["s_final"] == s
    assert eta <= 1e-15
    assert info_o["converged"] and abs(inf["iters"] - info_o["iters"]) <= 1
    # both solutions solve the same system to ~1e-15 backward error
    assert np.abs(X - Xo).max() <= 1e-12 * np.abs(Xo).max()


@pytest.mark.parametrize("nrhs", [1, 4, 5])
def test_precision_form_first_solve(nrhs):
    # with a tolerance every first solve meets, the precision form returns its
    # first solve: up to four right-hand sides it multiplies each diagonal
    # block by its inverse (ragged last block here: 1000 = 15 * 64 + 40), so
    # it agrees with the oracle's substitution on the same factors to
    # rounding; five take the substitution itself, bit for bit
    n, s = 1000, 6
    A = matgen.phi_matrix(n, n, 1.0, seed=27)
    B = matgen.uniform(n, nrhs, seed=28)
    Xg, inf = emu.dgesv_ir(emu.colmajor(A), emu.colmajor(B), nb=64, nslices=s, tol=1e300)
    assert inf["rc"] == 0 and inf["iters"] == 0 and inf["s_final"] == s
    LU, piv, info = O.getrf(A, nb=64, s=s)
    Xo = O.getrs(LU, piv, B)
    X = _host(Xg)
    if nrhs <= 4:
        assert np.abs(X - Xo).max() <= 1e-11 * np.abs(Xo).max()
    else:
        assert _same_bits(X, Xo)


def test_refinement_fallback_paths_match_oracle():
    A = matgen.phi_matrix(400, 400, 1.0, seed=23)
    B = matgen.uniform(400, 1, seed=24)
    Ag, Bg = emu.colmajor(A), emu.colmajor(B)
    try:
        emu.set_param("ir_force_fail", 1)
        _, inf = emu.dgesv_ir(Ag, Bg, nb=64, nslices=3)
        assert inf["rc"] == 0 and inf["s_final"] == 5
        emu.set_param("ir_force_fail", 2)
        _, inf = emu.dgesv_ir(Ag, Bg, nb=64, nslices=8)
        assert inf["rc"] == 1004 and inf["s_final"] == 9
    finally:
        emu.set_param("ir_force_fail", 0)
    _, io = O.gesv_ir(A, B, nb=64, s=3, force_fail=1)
    assert io["s_final"] == 5


def test_refinement_singular_reports_info():
    A = np.array(matgen.uniform(200, 200, seed=25), order="F")
    A[:, 50] = 0.0
    B = matgen.uniform(200, 1, seed=26)
    _, inf = emu.dgesv_ir(emu.colmajor(A), emu.colmajor(B), nb=64, nslices=5)
    assert inf["info"] == 51 and inf["rc"] == 0


# ------------------------------------------------------------ batched form

def _batch(count, seed, nmin=64, nmax=1024):
    specs = matgen.batched_specs(count, seed=seed, nmin=nmin, nmax=nmax)
    As = [matgen.phi_matrix(n, n, phi, seed=seed, substream=1000 + i)
          for i, (n, phi, r) in enumerate(specs)]
    Bs = [matgen.uniform(n, r, seed=seed, substream=5000 + i)
          for i, (n, phi, r) in enumerate(specs)]
    return specs, As, Bs


@pytest.mark.parametrize("nb,s", [(32, 5), (16, 3)])
def test_batched_solve_bit_exact_vs_oracle_and_single(nb, s):
    specs, As, Bs = _batch(12, seed=31, nmin=40, nmax=700)
    Ag = [emu.colmajor(a) for a in As]
    Bg = [emu.colmajor(b) for b in Bs]
    ipivs, info = emu.dgesv_batched(Ag, Bg, nb=nb, nslices=s)
    assert not _host(info).any()
    for i, (A, B) in enumerate(zip(As, Bs)):
        LU, piv, inf = O.getrf(A, nb=nb, s=s)
        X = O.getrs(LU, piv, B)
        assert np.array_equal(_host(ipivs[i]), piv), i
        assert _same_bits(_host(Ag[i]), LU), i
        assert _same_bits(_host(Bg[i]), X), i
        # grouped == single-system path with the same block size
        A1 = emu.colmajor(A)
        p1, _ = emu.dgetrf(A1, nb=nb, nslices=s)
        assert _same_bits(_host(A1), LU) and np.array_equal(_host(p1), piv)


def test_batched_solve_from_stored_factors():
    # factor once, solve two sets of right-hand sides from the stored factors;
    # sizes from 1 to the largest supported, ragged against the 32-column
    # panels and the 64-row solve blocks, one to eight right-hand sides
    sizes = [(1, 1), (2, 8), (63, 3), (64, 2), (65, 5), (300, 1), (1024, 4)]
    As = [matgen.phi_matrix(n, n, 1.5, seed=35, substream=1000 + i)
          for i, (n, r) in enumerate(sizes)]
    Bs = [matgen.uniform(n, r, seed=35, substream=5000 + i) for i, (n, r) in enumerate(sizes)]
    Ag = [emu.colmajor(a) for a in As]
    ipivs, info = emu.dgetrf_batched(Ag, nb=32, nslices=6)
    assert not _host(info).any()
    facts = [O.getrf(A, nb=32, s=6) for A in As]
    for rep in range(2):
        Bs2 = [b * (1.0 - 0.5 * rep) + rep for b in Bs]
        Bg = [emu.colmajor(b) for b in Bs2]
        emu.dgetrs_batched(Ag, ipivs, Bg)
        for i, (LU, piv, _) in enumerate(facts):
            assert np.array_equal(_host(ipivs[i]), piv), i
            assert _same_bits(_host(Bg[i]), O.getrs(LU, piv, Bs2[i])), (rep, i)
    # the same results as the factor-and-solve call
    Ag2 = [emu.colmajor(a) for a in As]
    Bg2 = [emu.colmajor(b) for b in Bs]
    emu.dgesv_batched(Ag2, Bg2, nb=32, nslices=6)
    Bg3 = [emu.colmajor(b) for b in Bs]
    emu.dgetrs_batched(Ag, ipivs, Bg3)
    for i in range(len(As)):
        assert _same_bits(_host(Bg3[i]), _host(Bg2[i])), i


def test_batched_graph_replay_with_new_matrices():
    specs, As, Bs = _batch(10, seed=32, nmin=30, nmax=500)
    for rep in range(3):
        # same shapes, new values: the cached graph is replayed
        As2 = [a * (1.0 + 0.25 * rep) + rep for a in As]
        Ag = [emu.colmajor(a) for a in As2]
        Bg = [emu.colmajor(b) for b in Bs]
        ipivs, info = emu.dgesv_batched(Ag, Bg, nb=32, nslices=4)
        torch.cuda.synchronize()
        for i in (0, 4, 9):
            LU, piv, _ = O.getrf(As2[i], nb=32, s=4)
            assert _same_bits(_host(Ag[i]), LU), (rep, i)
            assert _same_bits(_host(Bg[i]), O.getrs(LU, piv, Bs[i])), (rep, i)


def test_batched_singular_info_and_limits():
    specs, As, Bs = _batch(5, seed=33, nmin=50, nmax=200)
    A2 = np.array(As[2], order="F")
    A2[:, 7] = 0.0
    As[2] = A2
    Ag = [emu.colmajor(a) for a in As]
    ipivs, info = emu.dgetrf_batched(Ag, nb=32, nslices=5)
    h = _host(info)
    assert h[2] == 8 and h[[0, 1, 3, 4]].sum() == 0
    big = [emu.colmajor(np.eye(1100))]
    with pytest.raises(emu.EmuError):
        emu.dgetrf_batched(big, nb=32, nslices=5)


def test_batched_autotune_records_choice():
    specs, As, Bs = _batch(8, seed=34, nmin=64, nmax=400)
    Ag = [emu.colmajor(a) for a in As]
    Bg = [emu.colmajor(b) for b in Bs]
    nb, mult, ms = emu.autotune_batched(Ag, Bg, nslices=5)
    assert nb in (16, 32) and mult in (1, 2) and ms > 0
    # inputs untouched by tuning; nb = 0 then uses the tuned block size
    assert _same_bits(_host(Ag[3]), As[3])
    ipivs, info = emu.dgesv_batched(Ag, Bg, nb=0, nslices=5)
    LU, piv, _ = O.getrf(As[3], nb=nb, s=5)
    assert _same_bits(_host(Ag[3]), LU)
