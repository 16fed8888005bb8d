"""GPU parity and behaviour of the learned slice count (through the C ABI)."""
import numpy as np
import pytest
import torch

import matgen
import oracle as O
from oracle import learned as OL
import paper_2509_23565_amd as emu
from paper_2509_23565_amd import learned as L

pytestmark = pytest.mark.gpu


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_features_bit_exact():
    L21 = np.array(matgen.phi_matrix(700, 64, 4.0, seed=41), order="F")
    U12 = np.array(matgen.phi_matrix(64, 600, 4.0, seed=42), order="F")
    L21[::7, :] = 0.0
    L21[3, 5] = 0.0
    U12[:, 5] *= 2.0 ** -900
    U12[10, 100] = np.inf
    f = _host(emu.features(emu.colmajor(L21), emu.colmajor(U12)))
    assert np.array_equal(f.view(np.int32), OL.features(L21, U12).view(np.int32))


def test_mlp_gradient_matches_double_oracle():
    g = np.random.default_rng(43)
    p = emu.mlp_init(3)
    X = g.normal(size=(3000, 16)).astype(np.float32)
    y = g.integers(0, 7, size=3000).astype(np.int32)
    gg = _host(emu.mlp_grad(p, torch.as_tensor(X, device="cuda"), torch.as_tensor(y, device="cuda")))
    go = OL.mlp_grad(_host(p).astype(np.float64), X.astype(np.float64), y)
    assert np.linalg.norm(gg - go) <= 1e-4 * np.linalg.norm(go)
    prob, s = emu.mlp_infer(p, torch.as_tensor(X, device="cuda"))
    po, _ = OL.mlp_forward(_host(p).astype(np.float64), X.astype(np.float64))
    assert np.abs(_host(prob) - po).max() <= 1e-5
    c = np.cumsum(po, axis=1)
    clear = (np.abs(c - 0.95) > 1e-4).all(axis=1)
    assert np.array_equal(_host(s)[clear], OL.decode(po)[clear])


def test_tile_labels_match_oracle():
    A = matgen.phi_matrix(900, 900, 6.0, seed=44)
    LU, piv, _ = O.getrf(A, nb=128, s=9)
    L21, U12 = np.asfortranarray(LU[128:, :128]), np.asfortranarray(LU[:128, 128:])
    lab = _host(emu.tile_labels(emu.colmajor(L21), emu.colmajor(U12)))
    ref = OL.tile_labels(L21, U12)
    assert np.array_equal(lab, ref)


def test_training_reduces_loss_on_emulator_data():
    mats = [emu.colmajor(matgen.phi_matrix(1024, 1024, phi, seed=45 + i))
            for i, phi in enumerate((2.0, 6.0, 10.0))]
    X, y = L.training_set(mats, nb=256)
    assert len(set(_host(y).tolist())) >= 2
    p, hist = L.train(X, y, steps=300, lr=3e-3)
    print("training loss", [round(h, 4) for h in hist])
    assert hist[-1] < 0.7 * hist[0]


def _trained_params():
    mats = [emu.colmajor(matgen.phi_matrix(1024, 1024, phi, seed=50 + i))
            for i, phi in enumerate((1.0, 4.0, 8.0, 12.0))]
    X, y = L.training_set(mats, nb=256)
    p, _ = L.train(X, y, steps=300, lr=3e-3)
    return p


@pytest.mark.parametrize("m,n,nb,lookahead", [(800, 800, 128, 1), (800, 800, 128, 0),
                                               (600, 900, 128, 1), (900, 600, 128, 1),
                                               (700, 700, 256, 1)])
def test_adaptive_lu_bit_exact_given_its_maps(m, n, nb, lookahead):
    # with look-ahead the tiles over the next panel are updated first and the
    # others on the side stream; every tile gets the same operations
    p = _trained_params()
    A = matgen.phi_matrix(m, n, 6.0, seed=60)
    Ag = emu.colmajor(A)
    emu.set_param("lu_lookahead", lookahead)
    try:
        ipiv, info, smaps, (used, full) = emu.dgetrf_adaptive(Ag, p, nb=nb, s_full=9)
    finally:
        emu.set_param("lu_lookahead", 1)
    steps, k = [], 0
    for j1 in range(nb, min(m, n), nb):
        t = ((m - j1 + 255) // 256) * ((n - j1 + 255) // 256)
        steps.append(np.array(smaps[k:k + t]))
        k += t
    assert k == len(smaps)
    LU, piv, inf = OL.getrf_tiles(A, nb, steps)
    assert np.array_equal(_host(ipiv), piv)
    got = _host(Ag)
    assert np.array_equal(got.view(np.int64), np.ascontiguousarray(LU).view(np.int64))
    assert 0 < used <= full


def test_learned_gain_with_refinement():
    # The maps target the full count's accuracy (tau = 2^-40 against s = 9),
    # so the adaptive LU must reach 1e-15 with at most two refinement steps,
    # without the full-count fallback, on clearly fewer slice products than
    # the full count.  A model that predicts s = 9 everywhere, or one whose
    # factors need the fallback, fails here.
    p = _trained_params()
    n = 1024
    A = matgen.phi_matrix(n, n, 5.0, seed=61)
    b = matgen.uniform(n, 1, seed=62)
    Ag = emu.colmajor(A)
    LUg = Ag.clone()
    ipiv, info, smaps, (used, full) = emu.dgetrf_adaptive(LUg, p, nb=256, s_full=9)
    Xg = emu.colmajor(b)
    emu.dgetrs(LUg, ipiv, Xg)
    rc, iters, berr = emu.refine(Ag, LUg, ipiv, emu.colmajor(b), Xg, tol=1e-15, maxiter=2)
    eta = O.backward_error(A, _host(Xg), b)
    ratio = used / full
    print(f"learned slice counts: {ratio:.3f} of the full-count products, {iters} "
          f"refinement steps, eta {eta:.2e} (rc {rc}), counts {np.bincount(smaps)}")
    assert int(_host(info)[0]) == 0
    assert rc == 0 and iters <= 2 and eta <= 1e-15
    assert ratio <= 0.9
