"""Pins of the learned-form oracle (features, MLP, Adam, labels, tiled LU)."""
import numpy as np
import pytest

import matgen
import oracle as O
from oracle import learned as OL


def _params(seed=0):
    g = np.random.default_rng(seed)
    return g.normal(0.0, 0.2, size=64 * 16 + 64 + 64 * 64 + 64 + 7 * 64 + 7)


def test_features_of_a_hand_built_tile():
    # L21: 2 x 3, U12: 3 x 2 with known exponents
    L21 = np.array([[1.0, 0.25, 0.0], [3.0, 3.0, 2.0 ** -20]], order="F")
    U12 = np.array([[1.0, 0.0], [2.0 ** -10, 0.0], [2.0 ** -80, 0.0]], order="F")
    # rows: e = 1,-1 -> rho 0,-2 ; row 2: e(3)=2, rho 0,0,-19-... frexp(2^-20)=-19 -> -21
    # column 0: e = 1, -9, -79 -> rho 0, -10, -80 ; column 1 empty
    rho = np.array([0, -2, 0, 0, -21, 0, -10, -80])
    f = OL.features(L21, U12)[0]
    assert f[0] == -80 and f[1] == 0
    assert np.isclose(f[2], rho.mean()) and np.isclose(f[3], rho.std())
    hist = np.bincount(np.minimum(11, (-rho) // 7), minlength=12) / rho.size
    assert np.allclose(f[4:], hist)
    assert np.isclose(f[4:].sum(), 1.0)


def test_features_invariant_to_row_and_column_powers_of_two():
    L21 = matgen.phi_matrix(300, 40, 3.0, seed=1)
    U12 = matgen.phi_matrix(40, 270, 3.0, seed=2)
    f = OL.features(L21, U12)
    L2 = L21 * (2.0 ** np.arange(-150, 150))[:, None]
    U2 = U12 * (2.0 ** np.arange(135, -135, -1))[None, :]
    assert np.array_equal(OL.features(L2, U2), f)
    assert f.shape == (4, 16)


def test_mlp_uniform_output_for_zero_weights_and_gradient_by_differences():
    p0 = np.zeros(5703)
    X = matgen.uniform(9, 16, seed=3)
    prob, _ = OL.mlp_forward(p0, X)
    assert np.allclose(prob, 1.0 / 7.0)
    p = _params(4)
    y = np.random.default_rng(5).integers(0, 7, size=9)
    g = OL.mlp_grad(p, X, y)
    idx = np.random.default_rng(6).choice(p.size, size=60, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (OL.mlp_loss(p + e, X, y) - OL.mlp_loss(p - e, X, y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8


def test_adam_first_step_moves_by_lr_against_the_gradient_sign():
    p = _params(7)
    g = np.random.default_rng(8).normal(size=p.size)
    p1, m, v = OL.adam_step(p, g, np.zeros_like(p), np.zeros_like(p), 1, lr=1e-3)
    # exactly -lr g / (|g| + eps): within lr eps / |g| of -lr sign(g)
    assert np.all(np.abs((p1 - p) + 1e-3 * np.sign(g)) <= 1e-3 * 1e-8 / np.abs(g) + 1e-15)


def test_decode_takes_the_smallest_confident_count():
    prob = np.array([[0.96, 0.04, 0, 0, 0, 0, 0], [0.5, 0.4, 0.06, 0.04, 0, 0, 0],
                     [0, 0, 0, 0, 0, 0.5, 0.5]])
    assert list(OL.decode(prob)) == [3, 5, 9]


def test_labels_are_the_first_exact_count_for_integer_operands():
    L21 = matgen.int_matrix(260, 8, 7, seed=9)
    U12 = matgen.int_matrix(8, 270, 7, seed=10)
    lab = OL.tile_labels(L21, U12, s_lo=3, s_hi=9)
    assert list(lab) == [3, 3, 3, 3]        # one digit already exact


def test_tiled_lu_reduces_to_plain_lu_with_a_constant_map():
    A = matgen.phi_matrix(600, 600, 1.0, seed=11)
    nb = 128
    steps = [((600 - j1 + 255) // 256) ** 2 for j1 in range(nb, 600, nb)]
    for s in (4, 9):
        LU, piv, _ = OL.getrf_tiles(A, nb, [np.full(t, s) for t in steps])
        LU2, piv2, _ = O.getrf(A, nb=nb, s=s)
        assert np.array_equal(piv, piv2) and np.array_equal(LU, LU2)


def test_labels_follow_the_digit_counts_of_integer_tiles():
    # Tile-row I of L21 holds integers below 2^(7 a_I) with one entry at
    # 2^(7 a_I) - 1 (so its rows need exactly a_I digits), tile-column J of
    # U12 integers below 2^(7 b_J) likewise.  The emulated product of such a
    # tile is exact exactly from s = a_I + b_J - 1 on (all pairs i <= a_I,
    # j <= b_J lie under t = s + 1, and the pair (a_I, b_J) is dropped one
    # count below), so with tau = 0 the label is max(a_I + b_J - 1, s_lo).
    a = [1, 2, 3]
    b = [3, 1]
    k = 20
    g = np.random.default_rng(12)
    rows = [256, 256, 100]
    cols = [256, 200]
    L21 = np.vstack([g.integers(-(2 ** (7 * ai)) + 1, 2 ** (7 * ai), size=(r, k))
                     for ai, r in zip(a, rows)]).astype(np.float64)
    U12 = np.hstack([g.integers(-(2 ** (7 * bj)) + 1, 2 ** (7 * bj), size=(k, c))
                     for bj, c in zip(b, cols)]).astype(np.float64)
    r0 = 0
    for ai, r in zip(a, rows):
        L21[r0:r0 + r, 0] = 2.0 ** (7 * ai) - 1
        r0 += r
    c0 = 0
    for bj, c in zip(b, cols):
        U12[0, c0:c0 + c] = 2.0 ** (7 * bj) - 1
        c0 += c
    L21, U12 = np.asfortranarray(L21), np.asfortranarray(U12)
    lab = OL.tile_labels(L21, U12, s_lo=1, s_hi=9, tau=0.0)
    want = [max(a[I] + b[J] - 1, 1) for J in range(2) for I in range(3)]
    assert list(lab) == want
    assert len(set(want)) >= 4          # the labels span several counts


def test_tiled_lu_puts_a_tile_error_where_the_map_says():
    # Step 0 updates a 800 x 500 trailing block (4 x 2 tiles of 256).  Only
    # tile (I, J) = (3, 0) gets one slice (error near 2^-7 of its entries),
    # every other tile and every later step nine.  Blocked elimination keeps
    # each update's error where it was made: PA - LU is large in the columns
    # of that tile (100 .. 355) and at rounding level elsewhere, so an index
    # that mixes up I and J (q = J + I tn gives tile (1, 1), columns 356 ..)
    # would show it.
    m, n, nb = 900, 600, 100
    A = np.array(matgen.phi_matrix(m, n, 0.5, seed=13), order="F")
    smaps = []
    for j1 in range(nb, min(m, n), nb):
        tm, tn = -(-(m - j1) // 256), -(-(n - j1) // 256)
        smaps.append(np.full(tm * tn, 9))
    assert len(smaps[0]) == 8
    smaps[0][3 + 0 * 4] = 1
    LU, piv, info = OL.getrf_tiles(A, nb, smaps)
    assert info == 0
    PA = A.copy()
    for c in range(min(m, n)):
        p = int(piv[c]) - 1
        if p != c:
            PA[[c, p], :] = PA[[p, c], :]
    L = np.tril(LU, -1)[:, :n] + np.eye(m, n)
    U = np.triu(LU)[:n, :]
    E = np.abs(PA - L @ U).max(axis=0) / np.abs(A).max()
    inside, outside = E[100:356], np.concatenate([E[:100], E[356:]])
    assert inside.max() > 1e-6 and outside.max() < 1e-12


def test_per_tile_counts_cannot_beat_one_count_once_refinement_is_used():
    # With FP64 refinement (two steps at most) one constant count meets 1e-15
    # here; the ideal per-tile map at a tolerance that still needs at most two
    # steps (tau = 2^-26) costs more products per tile than that count.  The
    # full record (n = 1024, five phi) is tests/golden/learned_ceiling.json.
    n, nb = 768, 256
    A = matgen.phi_matrix(n, n, 8.0, seed=61)
    b = matgen.uniform(n, 1, seed=62)
    best = None
    for s in range(3, 10):
        _, io = O.gesv_ir(A, b, nb=nb, s=s, tol=1e-15, maxiter=2, s_max=s)
        if io["converged"]:
            best = s
            break
    assert best is not None
    LU, piv, _ = O.getrf(A, nb=nb, s=9)
    labels = []
    for j1 in range(nb, n, nb):
        j0 = j1 - nb
        labels.append(OL.tile_labels(np.asfortranarray(LU[j1:, j0:j1]),
                                     np.asfortranarray(LU[j0:j1, j1:]), tau=2.0 ** -26))
    lab = np.concatenate(labels)
    assert np.mean(lab * (lab + 1) / 2) >= best * (best + 1) / 2
