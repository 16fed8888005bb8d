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
