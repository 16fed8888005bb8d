"""GPU checks of the LU and the precision form at the sizes the benchmark
times (n = 16384 with nb = 256, n = 32768 with nb = 512), where the oracle
cannot repeat the whole factorization; properties that hold at any size:

* with nine slices the emulated update is below FP64 rounding, so the LU
  and solve must have the backward error of an FP64 LU with partial
  pivoting: the residual of 256 sampled rows, evaluated by the oracle in
  double-double ([A_i, b_i] . [x; -1], one rounding), over
  ||A||_inf ||x||_inf + ||b||_inf, below n u / 8 (Gaussian elimination's
  backward error is bounded by a small multiple of n u times the growth
  factor; these U(-1, 1) systems measure 6e-15 at n = 16384 and 1.2e-14 at
  n = 32768, about 30 times below the threshold, while factors computed
  from wrong operands give errors many orders larger);
* the look-ahead (updates on a second stream) changes no bit of the factors;
* the precision form (three slices and FP64 refinement) reaches 1e-15 in
  the same double-double measure.

Inputs: U(-1, 1) entries from a seeded torch generator on the GPU.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2509_23565_amd as emu

pytestmark = pytest.mark.gpu


def _system(n, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    A = (torch.rand((n, n), generator=g, dtype=torch.float64, device="cuda") * 2 - 1)
    A = A.t().contiguous().t()                       # column-major
    b = (torch.rand((1, n), generator=g, dtype=torch.float64, device="cuda") * 2 - 1).t()
    return A, b.contiguous().t().contiguous().t()


def _sampled_eta(A, x, b, seed):
    rows = np.sort(np.random.default_rng(seed).choice(A.shape[0], size=256, replace=False))
    rd = torch.as_tensor(rows, device="cuda")
    Ab = np.asfortranarray(np.hstack([A[rd].cpu().numpy(), b[rd].cpu().numpy()]))
    xe = np.asfortranarray(np.vstack([x.cpu().numpy(), [[-1.0]]]))
    r = O.dgemm_dd(Ab, xe)
    nA = float(A.abs().sum(dim=1).max())
    return float(np.abs(r).max() / (nA * float(x.abs().max()) + float(b.abs().max())))


@pytest.mark.parametrize("n,nb", [(16384, 256), (32768, 512)])
def test_lu_full_size_backward_error(n, nb):
    A, b = _system(n, seed=n + nb)
    F = A.clone()
    ipiv, info = emu.dgetrf(F, nb=nb, nslices=9)
    x = b.clone()
    emu.dgetrs(F, ipiv, x)
    torch.cuda.synchronize()
    assert int(info.cpu()[0]) == 0
    assert emu.status() & (emu.EMU_STATUS_PANEL_WAIT | emu.EMU_STATUS_SOLVE_WAIT) == 0
    eta = _sampled_eta(A, x, b, seed=n)
    print(f"n={n} nb={nb} s=9: sampled eta {eta:.2e}")
    assert eta < n * O.EPS / 8
    del A, F, x


def test_lu_full_size_lookahead_changes_no_bit():
    n, nb = 16384, 256
    A, _ = _system(n, seed=7)
    F1, F2 = A.clone(), A.clone()
    p1, _ = emu.dgetrf(F1, nb=nb, nslices=3)
    try:
        emu.set_param("lu_lookahead", 0)
        p2, _ = emu.dgetrf(F2, nb=nb, nslices=3)
    finally:
        emu.set_param("lu_lookahead", 1)
    torch.cuda.synchronize()
    assert torch.equal(p1, p2)
    assert torch.equal(F1.view(torch.int64), F2.view(torch.int64))


def test_precision_form_full_size_reaches_1e15():
    n = 32768
    A, b = _system(n, seed=11)
    X, inf = emu.dgesv_ir(A, b, nb=512, nslices=3, tol=1e-15)
    assert inf["rc"] == 0 and inf["info"] == 0
    eta = _sampled_eta(A, X, b, seed=12)
    print(f"n={n} s=3 + IR: {inf['iters']} steps, s_final {inf['s_final']}, sampled eta {eta:.2e}")
    assert eta <= 1e-15
