"""Fourth-kind Chebyshev smoothing (paper Sec. 3.1, Algorithm 3).

``cheb4`` follows Algorithm 3 step by step. ``w4`` and ``w4_hat`` evaluate the
polynomials of Eq. chebyshev_4th_kind through the three-term recurrence that
follows it; they serve the pins in the tests.
"""
from __future__ import annotations

import numpy as np


def cheb4(apply_a, apply_m, b, x0, beta: float, k: int, x_is_zero: bool = False):
    """Algorithm 3: Chebyshev iteration of the fourth kind, degree k >= 1.

    apply_a(v) = A v, apply_m(v) = M v, beta >= lambda_max(MA).
    x_is_zero: x0 is zero, so the first residual is b itself.
    """
    if k < 1:
        raise ValueError("degree must be >= 1")
    x = np.zeros_like(b) if x_is_zero else np.array(x0, dtype=np.float64, copy=True)
    r = b.copy() if x_is_zero else b - apply_a(x)
    p = apply_m(r)
    mu = 1.0 / 3.0
    d = 4.0 / beta
    x = x + d * mu * p
    for _ in range(2, k + 1):
        r = b - apply_a(x)
        p = mu * mu * p + apply_m(r)
        mu = 1.0 / (2.0 - mu)
        x = x + d * mu * p
    return x


def w4(k: int, t):
    """W_k(t): W_0 = 1, W_1 = 2t + 1, W_{n+1} = 2t W_n - W_{n-1}."""
    t = np.asarray(t, dtype=np.float64)
    w_prev = np.ones_like(t)
    if k == 0:
        return w_prev
    w = 2.0 * t + 1.0
    for _ in range(1, k):
        w_prev, w = w, 2.0 * t * w - w_prev
    return w


def w4_hat(k: int, lam, beta: float):
    """W^_k(lambda) = W_k(1 - 2 lambda / beta) / (2k + 1) (Eq. chebyshev_4th_kind)."""
    return w4(k, 1.0 - 2.0 * np.asarray(lam, dtype=np.float64) / beta) / (2 * k + 1)


def cheb4_increment_form(apply_a, apply_m, b, x0, beta: float, k: int):
    """The same polynomial written as an increment recurrence.

    From the paper's parameters mu_n = (2n+1)/(2n+3) and mu_n mu_{n-1} =
    (2n-1)/(2n+3), Algorithm 3's update x += d mu_n p_n with p_n =
    mu_{n-1}^2 p_{n-1} + M r_n becomes, for delta_n = d mu_n p_n,
        delta_0 = (4 / (3 beta)) M r_0,
        delta_n = (2n-1)/(2n+3) delta_{n-1} + (8n+4)/((2n+3) beta) M r_n,
    with r_n = r_{n-1} - A delta_{n-1}. Used only as an independent
    cross-check of Algorithm 3.
    """
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - apply_a(x)
    delta = (4.0 / (3.0 * beta)) * apply_m(r)
    x = x + delta
    for n in range(1, k):
        r = r - apply_a(delta)
        delta = ((2 * n - 1) / (2 * n + 3)) * delta + ((8 * n + 4) / ((2 * n + 3) * beta)) * apply_m(r)
        x = x + delta
    return x


def cheb4_spectral(gmat: np.ndarray, amat: np.ndarray, b, x0, beta: float, k: int):
    """Plain definition of the smoother for tiny dense problems.

    A polynomial iteration satisfies x_k = x0 + q_{k-1}(MA) M r_0 with
    p_k(t) = 1 - t q_{k-1}(t) (Eq. polynomial_iteration_x, preconditioned), and
    p_k = W^_k. With M = G^T G, q(MA) M = G^T q(G A G^T) G, so
    x_k = x0 + G^T V diag(q(lambda)) V^T G r_0 with G A G^T = V Lambda V^T.
    """
    bmat = gmat @ amat @ gmat.T
    bmat = 0.5 * (bmat + bmat.T)
    lam, v = np.linalg.eigh(bmat)
    q = (1.0 - w4_hat(k, lam, beta)) / lam
    r0 = b - amat @ x0
    return x0 + gmat.T @ (v @ (q * (v.T @ (gmat @ r0))))
