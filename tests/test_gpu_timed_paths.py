"""GPU parity of the kernel variants that the benchmark runs at full size.

Each case is the smallest shape that takes the same kernel variant as a
timed workload, compared with the CPU oracle bit for bit:

* the emulated GEMM at s = 9 with K between the plain exact length (14784)
  and the split-diagonal one (16640): the longest diagonal is split over two
  accumulator tiles and folded back in the epilogue (the 16384^3 product);
* tile counts that are multiples of 16 in both directions (every square
  size the benchmark times), where the workgroups of all XCDs share one
  block of tiles at a time ("gemm_map" 1, the default), against the oracle
  and against the per-XCD order;
* K above 16640: exact-length chunks of INT32 partial sums, added in INT64
  and recombined into C by the combine pass;
* the batched LU at s = 6, 7 and 9 (the pipelined one-K-step grouped GEMM)
  with systems up to n = 1024;
* tall LU panels: leaves of 9 and 17 workgroups, and in-panel updates that
  take the 64- and 32-row order-preserving tiles (n = 32768, nb = 512 runs
  these);
* three Adam steps of the MLP, each from the library's own state, against
  the oracle's step on the oracle's gradient.
"""
import numpy as np
import pytest
import torch

import matgen
import oracle as O
from oracle import learned as OL
import paper_2509_23565_amd as emu

pytestmark = pytest.mark.gpu


def _same_bits(a, b):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64))
    return a.shape == b.shape and np.array_equal(a.view(np.int64), b.view(np.int64))


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


# exact INT32 lengths (multiples of 32) for the longest slot of s = 9, t = 10:
# nine pairs -> 14784, eight pairs (longest diagonal split) -> 16640
K_PLAIN_S9 = 14784
K_SPLIT_S9 = 16640


@pytest.mark.parametrize("m,n,k,s", [(1024, 2048, 300, 9), (2048, 2048, 200, 3)])
def test_dgemm_shared_tile_block_order(m, n, k, s):
    A = matgen.phi_matrix(m, k, 1.0, seed=74, substream=0)
    B = matgen.phi_matrix(k, n, 1.0, seed=74, substream=1)
    Ag, Bg = emu.colmajor(A), emu.colmajor(B)
    ref = O.dgemm_emu(A, B, s)
    try:
        for mp in (1, 0):
            emu.set_param("gemm_map", mp)
            Cg = emu.dgemm(Ag, Bg, nslices=s)
            assert _same_bits(_host(Cg), ref), mp
    finally:
        emu.set_param("gemm_map", 1)


def test_dgemm_split_longest_diagonal_s9():
    m, n, k = 200, 300, 16000
    assert K_PLAIN_S9 < k <= K_SPLIT_S9
    A = matgen.phi_matrix(m, k, 1.0, seed=71, substream=0)
    B = matgen.phi_matrix(k, n, 1.0, seed=71, substream=1)
    C0 = matgen.uniform(m, n, seed=71, substream=2)
    Ag, Bg = emu.colmajor(A), emu.colmajor(B)
    for alpha, beta in ((1.0, 0.0), (-0.7, 1.3)):
        Cg = emu.colmajor(C0)
        emu.dgemm(Ag, Bg, Cg, alpha=alpha, beta=beta, nslices=9)
        ref = O.dgemm_emu(A, B, 9, alpha=alpha, beta=beta, C=C0)
        assert _same_bits(_host(Cg), ref), (alpha, beta)


@pytest.mark.parametrize("extreme", [False, True])
def test_dgemm_chunked_combine_into_c(extreme):
    m, n, k = 70, 90, 20000
    assert k > K_SPLIT_S9
    if extreme:
        # every digit 127: true diagonal sums exceed 2^31, so the INT64 fold
        # across chunks is needed
        x = 1.0 - 2.0 ** -53
        A = np.full((m, k), x, order="F")
        A[::2, :] *= -1.0
        B = np.full((k, n), x, order="F")
        B[:, 1::3] *= -1.0
    else:
        A = matgen.phi_matrix(m, k, 2.0, seed=72, substream=0)
        B = matgen.phi_matrix(k, n, 2.0, seed=72, substream=1)
    C0 = matgen.uniform(m, n, seed=72, substream=2)
    Cg = emu.colmajor(C0)
    emu.dgemm(emu.colmajor(A), emu.colmajor(B), Cg, alpha=1.5, beta=-0.5, nslices=9)
    ref, parts = O.dgemm_emu(A, B, 9, alpha=1.5, beta=-0.5, C=C0, return_parts=True)
    assert _same_bits(_host(Cg), ref)
    if extreme:
        assert max(np.abs(parts["D"][g]).max() for g in range(2, 11)) > 2 ** 31


@pytest.mark.parametrize("s", [6, 7, 9])
def test_batched_pipelined_grouped_gemm(s):
    sizes = [1024, 777, 513, 300, 64]
    As = [matgen.phi_matrix(n, n, 2.0, seed=73, substream=i) for i, n in enumerate(sizes)]
    Bs = [matgen.uniform(n, 1 + i % 3, seed=73, substream=100 + i)
          for i, n in enumerate(sizes)]
    Ag = [emu.colmajor(a) for a in As]
    Bg = [emu.colmajor(b) for b in Bs]
    ipivs, info = emu.dgesv_batched(Ag, Bg, nb=32, nslices=s)
    assert not _host(info).any()
    for i, (A, B) in enumerate(zip(As, Bs)):
        LU, piv, inf = O.getrf(A, nb=32, s=s)
        assert np.array_equal(_host(ipivs[i]), piv), i
        assert _same_bits(_host(Ag[i]), LU), i
        assert _same_bits(_host(Bg[i]), O.getrs(LU, piv, B)), i


@pytest.mark.parametrize("m,n,nb,s", [(16640, 520, 512, 3), (33000, 32, 32, 3)])
def test_getrf_tall_leaves_and_wide_tiles(m, n, nb, s):
    # 16640 rows: leaves of 9 workgroups, in-panel updates of 16384 x 256
    # (64-row tiles) and 16512 x 128 (32-row tiles); 33000 rows: 17 workgroups
    A = matgen.phi_matrix(m, n, 1.0, seed=74)
    Ag = emu.colmajor(A)
    emu.status()
    ipiv, info = emu.dgetrf(Ag, nb=nb, nslices=s)
    assert emu.status() == 0
    LU, piv, inf = O.getrf(A, nb=nb, s=s)
    assert int(_host(info)[0]) == inf
    assert np.array_equal(_host(ipiv), piv)
    assert _same_bits(_host(Ag), LU)


def test_adam_steps_match_oracle():
    # each step from the GPU's own state (parameters and moments), so the
    # comparison isolates one step: the oracle's gradient at those
    # parameters and its Adam update against the library's kernels
    g = np.random.default_rng(75)
    p = emu.mlp_init(5)
    X = g.normal(size=(2000, 16)).astype(np.float32)
    y = g.integers(0, 7, size=2000).astype(np.int32)
    Xg = torch.as_tensor(X, device="cuda")
    yg = torch.as_tensor(y, device="cuda")
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    lr = 1e-3
    for step in (1, 2, 3):
        p0, m0, v0 = (_host(t).astype(np.float64) for t in (p, m, v))
        go = OL.mlp_grad(p0, X.astype(np.float64), y)
        po, mo, vo = OL.adam_step(p0, go, m0, v0, step, lr=lr)
        emu.mlp_train_step(p, Xg, yg, m, v, step, lr=lr)
        # moments: norm-wise against the oracle's (FP32 gradient vs double)
        assert np.linalg.norm(_host(m) - mo) <= 1e-4 * np.linalg.norm(mo), step
        assert np.linalg.norm(_host(v) - vo) <= 1e-4 * np.linalg.norm(vo), step
        # the update itself where the gradient is well above the FP32
        # gradient's error (there the step's direction is not in doubt)
        dg = _host(p).astype(np.float64) - p0
        do = po - p0
        sure = np.abs(go) >= 1e-3 * np.abs(go).max()
        assert sure.mean() > 0.5
        assert np.abs(dg[sure] - do[sure]).max() <= 1e-3 * lr, step


def test_batched_grouped_tile_shapes_and_tuner():
    # the 64 x 64 grouped tile (four waves) against the default 64 x 128, and
    # the oracle; then the autotuner's choice over block size, grid and tile
    specs = matgen.batched_specs(10, seed=35, nmax=600)
    As = [matgen.phi_matrix(n, n, phi, seed=35, substream=1000 + i)
          for i, (n, phi, r) in enumerate(specs)]
    Bs = [matgen.uniform(n, r, seed=35, substream=5000 + i) for i, (n, phi, r) in enumerate(specs)]
    for s in (7, 9):
        outs = []
        try:
            for tile in (0, 1):
                emu.set_param("batched_tile", tile)
                Ag = [emu.colmajor(a) for a in As]
                Bg = [emu.colmajor(b) for b in Bs]
                emu.dgesv_batched(Ag, Bg, nb=32, nslices=s)
                outs.append(([_host(a) for a in Ag], [_host(b) for b in Bg]))
        finally:
            emu.set_param("batched_tile", 0)
        for i in range(len(As)):
            assert _same_bits(outs[0][0][i], outs[1][0][i]) and _same_bits(outs[0][1][i], outs[1][1][i])
        for i in (0, 4):
            LU, piv, _ = O.getrf(As[i], nb=32, s=s)
            assert _same_bits(outs[1][0][i], LU)
            assert _same_bits(outs[1][1][i], O.getrs(LU, piv, Bs[i]))
    Ag = [emu.colmajor(a) for a in As]
    Bg = [emu.colmajor(b) for b in Bs]
    nb, mult, ms, tile = emu.autotune_batched(Ag, Bg, nslices=7, with_tile=True)
    assert nb in (16, 32) and mult in (1, 2) and tile in (0, 1) and ms > 0
    emu.dgesv_batched(Ag, Bg, nb=0, nslices=7)
    LU, piv, _ = O.getrf(As[2], nb=nb, s=7)
    assert _same_bits(_host(Ag[2]), LU)
