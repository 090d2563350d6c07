"""Learned pattern proposer driver: assembles training sets and trains the
network through the C ABI (features, labels, training and proposal all run
in the library's kernels; torch only holds device buffers)."""
from __future__ import annotations

import torch

from . import binding as chf


def dataset(items, device="cuda"):
    """items: iterable of (A, nx, ny, P) with P the target pattern (Algorithm
    1's). Returns (features float32 [n, 6], labels float32 [n]) on the device."""
    feats, labels = [], []
    for A, nx, ny, P in items:
        rowptr, _ = chf.mlp_candidates(A)
        n = int(rowptr[-1])
        f = torch.empty(n * chf.NFEAT, dtype=torch.float32, device=device)
        y = torch.empty(n, dtype=torch.float32, device=device)
        chf.mlp_features(A, nx, ny, f)
        chf.mlp_labels(A, P, y)
        feats.append(f)
        labels.append(y)
    return torch.cat(feats).view(-1, chf.NFEAT), torch.cat(labels)


def train(X, Y, params0, perm, epochs=4, batch=8192, lr=2e-3):
    """Mini-batch Adam over the rows of (X, Y) in the order of `perm`."""
    net = chf.mlp_create(params0)
    hist = chf.mlp_train(net, X, Y, Y.shape[0], perm, batch=batch, epochs=epochs, lr=lr)
    return net, hist


def template_offsets(prow, pcol, nx, ny, k):
    """Grid offsets (dx, dy, dz) of the off-diagonal blocks of row k of a
    pattern on an nx x ny (x nz) patch grid, for chf_pattern_template."""
    def coords(i):
        return i % nx, (i // nx) % ny, i // (nx * ny)
    kx, ky, kz = coords(int(k))
    out = []
    for c in pcol[prow[k]:prow[k + 1]]:
        c = int(c)
        if c != k:
            cx, cy, cz = coords(c)
            out.append((cx - kx, cy - ky, cz - kz))
    return out

