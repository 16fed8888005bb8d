"""Training-data generation and training loop for the learned slice count.

Host-side orchestration only: every computation runs in libemu (LU factors,
features, emulator-produced labels, MLP training kernels).

Samples are the 256 x 256 tiles of the Schur updates of emulated LUs: for a
factored matrix the operands of step j are L21 = LU[j1:, j0:j1] and
U12 = LU[j0:j1, j1:] (rows of L21 in their final interchange order).  A
tile's label is the smallest slice count whose emulated product of those
operands agrees with the full-count product within tau (emu_tile_labels).
"""
from __future__ import annotations

from . import dgetrf, features, mlp_init, mlp_train_step, tile_labels


def training_set(mats, nb=256, s_lo=3, s_hi=9, tau=2.0 ** -40, max_steps=None):
    """Features (float32 [N][16]) and classes (int32 [N], s - 3) on the GPU."""
    import torch
    Xs, ys = [], []
    for A in mats:
        LU = A.clone()
        dgetrf(LU, nb=nb, nslices=s_hi)
        n = LU.shape[0]
        steps = 0
        for j0 in range(0, n - nb, nb):
            j1 = j0 + nb
            if j1 >= n:
                break
            L21 = LU[j1:, j0:j1]
            U12 = LU[j0:j1, j1:]
            Xs.append(features(L21, U12))
            ys.append(tile_labels(L21, U12, s_lo, s_hi, tau) - 3)
            steps += 1
            if max_steps and steps >= max_steps:
                break
    return torch.cat(Xs), torch.cat(ys).to(torch.int32)


def train(X, y, steps=400, lr=3e-3, seed=0):
    """Full-batch Adam on the mean cross-entropy; returns (params, losses)."""
    import torch
    p = mlp_init(seed, device=X.device)
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    loss = torch.zeros(X.shape[0], dtype=torch.float32, device=X.device)
    hist = []
    for k in range(1, steps + 1):
        mlp_train_step(p, X, y, m, v, k, lr=lr, loss=loss)
        if k == 1 or k == steps or k % 50 == 0:
            hist.append(float(loss.mean()))
    return p, hist
