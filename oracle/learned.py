"""Oracle for the learned slice-count part.  TEST INFRASTRUCTURE ONLY.

Written from the definitions (the learned form is not in the paper; its
features measure the digit loss of the paper's eqn (3): how far an element's
exponent sits below the largest exponent of its row or column):

* features of tile (I, J) of the update C = L21 U12: rho over the nonzero
  finite elements of L21's rows of block I (relative to each row's largest
  frexp exponent) and U12's columns of block J (relative to each column's);
  [min, max, mean, std, 12 bin fractions of -rho with bins of width 7, the
  last open-ended], computed in double and rounded to float32;
* the MLP 16 -> 64 -> 64 -> 7 (ReLU, softmax) in double, its mean
  cross-entropy, its gradient by the chain rule, and one Adam step;
* tile labels: smallest s whose emulated product is within tau of the
  s_hi product (relative Frobenius norm per tile);
* LU whose update uses a given slice count per 256 x 256 tile.
"""
from __future__ import annotations

import numpy as np

from . import emu as E

FT = 256
NBIN = 12
H = 64
NCLS = 7


def _frexp_exp(x):
    return np.frexp(x)[1].astype(np.int64)


def _line_stats(X, axis):
    """Per line (axis=1: rows, 0: columns): list of rho arrays."""
    X = np.asarray(X, dtype=np.float64)
    good = (X != 0.0) & np.isfinite(X)
    e = np.where(good, _frexp_exp(np.where(good, X, 1.0)), np.iinfo(np.int64).min)
    emax = e.max(axis=axis, initial=np.iinfo(np.int64).min)
    rho = e - (emax[:, None] if axis == 1 else emax[None, :])
    return rho, good


def features(L21, U12):
    """float32 array [tiles][16], tile index I + J * tiles_m."""
    L21 = np.asarray(L21, dtype=np.float64)
    U12 = np.asarray(U12, dtype=np.float64)
    m, n = L21.shape[0], U12.shape[1]
    tm, tn = (m + FT - 1) // FT, (n + FT - 1) // FT
    rL, gL = _line_stats(L21, axis=1)
    rU, gU = _line_stats(U12, axis=0)
    out = np.zeros((tm * tn, 16), dtype=np.float32)
    for J in range(tn):
        cu = rU[:, J * FT:(J + 1) * FT][gU[:, J * FT:(J + 1) * FT]]
        for I in range(tm):
            rl = rL[I * FT:(I + 1) * FT, :][gL[I * FT:(I + 1) * FT, :]]
            rho = np.concatenate([rl, cu]).astype(np.int64)
            f = out[I + J * tm]
            if rho.size == 0:
                continue
            c = float(rho.size)
            mean = float(rho.sum()) / c
            var = float((rho * rho).sum()) / c - mean * mean
            f[0] = np.float32(rho.min())
            f[1] = np.float32(rho.max())
            f[2] = np.float32(mean)
            f[3] = np.float32(np.sqrt(var if var > 0.0 else 0.0))
            bins = np.minimum(NBIN - 1, (-rho) // 7)
            hist = np.bincount(bins, minlength=NBIN)
            f[4:] = (hist / c).astype(np.float32)
    return out


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * 16].reshape(H, 16); o += H * 16
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + NCLS * H].reshape(NCLS, H); o += NCLS * H
    b3 = p[o:o + NCLS]; o += NCLS
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def mlp_forward(p, X):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W3.T + b3
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    prob = e / e.sum(axis=1, keepdims=True)
    return prob, (X, a1, h1, a2, h2)


def mlp_loss(p, X, y):
    prob, _ = mlp_forward(p, X)
    return float(-np.log(prob[np.arange(len(y)), y]).mean())


def mlp_grad(p, X, y):
    """Gradient of the mean cross-entropy (same layout as the parameters)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    prob, (X, a1, h1, a2, h2) = mlp_forward(p, X)
    B = X.shape[0]
    d3 = prob.copy()
    d3[np.arange(B), y] -= 1.0
    d3 /= B
    gW3 = d3.T @ h2
    gb3 = d3.sum(axis=0)
    d2 = (d3 @ W3) * (a2 > 0)
    gW2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (a1 > 0)
    gW1 = d1.T @ X
    gb1 = d1.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def adam_step(p, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def decode(prob, conf=0.95):
    """Smallest s whose cumulative class probability reaches conf."""
    c = np.cumsum(prob, axis=1)
    idx = np.argmax(c >= conf, axis=1)
    idx = np.where((c >= conf).any(axis=1), idx, NCLS - 1)
    return 3 + np.minimum(idx, NCLS - 1)


def tile_labels(L21, U12, s_lo=3, s_hi=9, tau=2.0 ** -40):
    m, n = L21.shape[0], U12.shape[1]
    tm, tn = (m + FT - 1) // FT, (n + FT - 1) // FT
    Xr = E.dgemm_emu(L21, U12, s_hi)
    lab = np.full(tm * tn, s_hi, dtype=np.int64)
    done = np.zeros(tm * tn, bool)
    for s in range(s_lo, s_hi):
        Xs = E.dgemm_emu(L21, U12, s)
        for J in range(tn):
            for I in range(tm):
                q = I + J * tm
                if done[q]:
                    continue
                sl = (slice(I * FT, (I + 1) * FT), slice(J * FT, (J + 1) * FT))
                err = np.linalg.norm(Xs[sl] - Xr[sl])
                ref = np.linalg.norm(Xr[sl])
                if err <= tau * ref:
                    lab[q] = s
                    done[q] = True
    return lab


def getrf_tiles(A, nb, smaps):
    """Blocked LU whose step-k update uses slice count smaps[k][q] on the
    256 x 256 tile q = I + J * tiles_m of A22 (FP64 panel/laswp/TRSM as in
    emu.getrf).  smaps: list of per-step arrays, steps with an update only."""
    LU = np.array(A, dtype=np.float64, order="F", copy=True)
    m, n = LU.shape
    mn = min(m, n)
    ipiv = np.zeros(mn, dtype=np.int64)
    info = 0
    step = 0
    for j0 in range(0, mn, nb):
        jb = min(nb, mn - j0)
        j1 = j0 + jb
        pinfo = E.getf2(LU[j0:, j0:j1], ipiv, j0)
        if info == 0 and pinfo:
            info = pinfo
        for c in range(j0, j1):
            p = int(ipiv[c]) - 1
            if p != c:
                LU[[c, p], :j0] = LU[[p, c], :j0]
                LU[[c, p], j1:] = LU[[p, c], j1:]
        if j1 < n:
            E.trsm_unit_lower(LU[j0:j1, j0:j1], LU[j0:j1, j1:])
            if j1 < m:
                M, N = m - j1, n - j1
                tm = (M + FT - 1) // FT
                smap = smaps[step]
                step += 1
                L21 = LU[j1:, j0:j1].copy(order="F")
                U12 = LU[j0:j1, j1:].copy(order="F")
                for q, s in enumerate(smap):
                    I, J = q % tm, q // tm
                    r = slice(j1 + I * FT, j1 + min(M, (I + 1) * FT))
                    c = slice(j1 + J * FT, j1 + min(N, (J + 1) * FT))
                    LU[r, c] = E.dgemm_emu(L21[I * FT:(I + 1) * FT, :],
                                           U12[:, J * FT:(J + 1) * FT], int(s),
                                           alpha=-1.0, beta=1.0, C=LU[r, c])
    return LU, ipiv, info
