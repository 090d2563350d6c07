"""Learned pattern proposer: features, the 4-64-64-1 ReLU network and its
gradient in FP64 (test infrastructure for the GPU kernels).

Features of candidate c for block row k (c in the strictly lower part of the
row pattern of A^2):
  f0 = ||A_kc||_F / sqrt(||A_kk||_F ||A_cc||_F)
  f1 = ||A_cc^{-1} A_ck||_F
  f2, f3, f4 = signed patch offset (dx, dy, dz) of c from k on the grid
  f5 = one-step gain -log rho_c with P_k = {k} (Lemma 2.4)
Label: c belongs to the final pattern of Algorithm 1. Loss: mean binary
cross-entropy with logits. Parameter layout (4673 values): W1[64][6], b1[64],
W2[64][64], b2[64], W3[64], b3.
"""
from __future__ import annotations

import numpy as np

from . import adaptive
from .bsr import Bsr

H, NIN = 64, 6
NPARAM = H * NIN + H + H * H + H + H + 1


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    w1 = p[o:o + H * NIN].reshape(H, NIN)
    o += H * NIN
    b1 = p[o:o + H]
    o += H
    w2 = p[o:o + H * H].reshape(H, H)
    o += H * H
    b2 = p[o:o + H]
    o += H
    w3 = p[o:o + H]
    b3 = p[o + H]
    return w1, b1, w2, b2, w3, b3


def forward(p, x):
    w1, b1, w2, b2, w3, b3 = unpack(p)
    z1 = x @ w1.T + b1
    h1 = np.maximum(z1, 0)
    z2 = h1 @ w2.T + b2
    h2 = np.maximum(z2, 0)
    return h2 @ w3 + b3, (x, z1, h1, z2, h2)


def loss(p, x, y):
    z, _ = forward(p, x)
    return float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def loss_grad(p, x, y):
    """Mean BCE-with-logits and its gradient by backpropagation."""
    w1, b1, w2, b2, w3, b3 = unpack(p)
    z, (x, z1, h1, z2, h2) = forward(p, x)
    n = x.shape[0]
    lval = float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / n
    g_w3 = h2.T @ dz
    g_b3 = dz.sum()
    d2 = np.outer(dz, w3) * (z2 > 0)
    g_w2 = d2.T @ h1
    g_b2 = d2.sum(0)
    d1 = (d2 @ w2) * (z1 > 0)
    g_w1 = d1.T @ x
    g_b1 = d1.sum(0)
    g = np.concatenate([g_w1.ravel(), g_b1, g_w2.ravel(), g_b2, g_w3, [g_b3]])
    return lval, g


def adam_step(p, g, m, v, t: int, lr: float, beta1: float, beta2: float, eps: float):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1), step t >= 1, in
    FP64: first and second moment estimates, their bias corrections by
    1 - beta^t, and the parameter move lr * m_hat / (sqrt(v_hat) + eps).
    Returns the new (p, m, v). The network's optimiser; not in the paper."""
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return np.asarray(p, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps), m, v


def a2_candidates(a: Bsr):
    """Strictly lower part of the row pattern of A^2, rows ascending."""
    rowptr, cols = [0], []
    for k in range(a.nb):
        s = set()
        for j in a.cols(k):
            for c in a.cols(int(j)):
                if c < k:
                    s.add(int(c))
        cols.extend(sorted(s))
        rowptr.append(len(cols))
    return np.array(rowptr, dtype=np.int64), np.array(cols, dtype=np.int64)


def features(a: Bsr, nx: int, ny: int, rows=None):
    crow, ccol = a2_candidates(a)
    rows = range(a.nb) if rows is None else rows
    out = {}
    for k in rows:
        akk = a.block(k, k)
        kx, ky, kz = k % nx, (k // nx) % ny, k // (nx * ny)
        cand = [int(c) for c in ccol[crow[k]:crow[k + 1]]]
        g = adaptive.gains(a, k, [k], cand) if cand else []
        f = []
        for c, gc in zip(cand, g):
            akc, acc = a.block(k, c), a.block(c, c)
            cx, cy, cz = c % nx, (c // nx) % ny, c // (nx * ny)
            f.append([np.linalg.norm(akc) / np.sqrt(np.linalg.norm(akk) * np.linalg.norm(acc)),
                      np.linalg.norm(np.linalg.solve(acc, akc.T)),
                      cx - kx, cy - ky, cz - kz,
                      gc])
        out[int(k)] = (np.array(cand, dtype=np.int64), np.array(f).reshape(-1, NIN))
    return crow, ccol, out


def labels(crow, ccol, prow, pcol):
    """1 where the candidate is in the row's final adaptive pattern."""
    y = np.zeros(len(ccol))
    for k in range(len(crow) - 1):
        chosen = set(int(c) for c in pcol[prow[k]:prow[k + 1]])
        for e in range(crow[k], crow[k + 1]):
            y[e] = 1.0 if int(ccol[e]) in chosen else 0.0
    return y


def topk_pattern(crow, ccol, score, t: int):
    """t best candidates per row (ties to the smaller column) plus the diagonal."""
    prow, pcol = [0], []
    for k in range(len(crow) - 1):
        idx = list(range(crow[k], crow[k + 1]))
        idx.sort(key=lambda e: (-score[e], ccol[e]))
        row = sorted([int(ccol[e]) for e in idx[:t]] + [k])
        pcol.extend(row)
        prow.append(len(pcol))
    return np.array(prow, dtype=np.int64), np.array(pcol, dtype=np.int64)
