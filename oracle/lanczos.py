"""Largest eigenvalue of the FSAI-preconditioned operator by Lanczos (Sec. 5,
opening paragraphs: 100 Lanczos iterations, estimate multiplied by 1.01).

The operator is G A G^T, which has the spectrum of M A = G^T G A. Plain
three-term recurrence without reorthogonalisation; the start vector is given
by the caller (seeded N(0,1)). The Ritz value comes from LAPACK's symmetric
tridiagonal eigensolver. The number of steps is min(iters, N); the iteration
stops early when beta_j < 1e-12 * max |alpha|.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import eigh_tridiagonal


def lanczos_tridiag(apply_op, v0, iters: int = 100):
    n = v0.shape[0]
    m = min(iters, n)
    v = v0 / np.linalg.norm(v0)
    v_prev = np.zeros_like(v)
    beta_prev = 0.0
    alphas, betas = [], []
    for j in range(m):
        w = apply_op(v)
        alpha = float(v @ w)
        w = w - alpha * v - beta_prev * v_prev
        beta = float(np.linalg.norm(w))
        alphas.append(alpha)
        if j == m - 1:
            break
        if beta < 1e-12 * max(abs(x) for x in alphas):
            break
        betas.append(beta)
        v_prev, v = v, w / beta
        beta_prev = beta
    return np.array(alphas), np.array(betas)


def lmax(apply_op, v0, iters: int = 100, safety: float = 1.01):
    """Returns (safety * theta_max, theta_max)."""
    alphas, betas = lanczos_tridiag(apply_op, v0, iters)
    if len(alphas) == 1:
        theta = alphas[0]
    else:
        theta = float(eigh_tridiagonal(alphas, betas, eigvals_only=True)[-1])
    return safety * theta, theta
