"""Polynomial smoothers of Sec. 3: fourth-kind Chebyshev (Algorithm 3), and
the comparators of Sec. 3.1, first-kind Chebyshev (Algorithm 2) and
Richardson smoothing S = (I - omega M A)^k.

``cheb4``, ``cheb1`` and ``richardson`` derive each algorithm's per-step
coefficients first and then run one shared increment loop.
``w4`` and ``w4_hat`` evaluate the polynomials of Eq. chebyshev_4th_kind
through the three-term recurrence that follows it; ``t1_hat`` evaluates
Eq. chebyshev_1st_kind with NumPy's Chebyshev series. They serve the pins in
the tests, together with ``poly_spectral`` (the smoother written as the
polynomial of MA it applies).
"""
from __future__ import annotations

import numpy as np


def _polynomial_smoother(apply_a, apply_m, b, x0, carry, scale, x_is_zero: bool):
    """Shared driver of the polynomial smoothers of Sec. 3.

    Every smoother here moves x by an increment that mixes the previous
    increment with the preconditioned residual of the current iterate:
        z_i = M (b - A x_{i-1}),
        delta_i = carry[i] delta_{i-1} + scale[i] z_i   (carry[0] unused),
        x_i = x_{i-1} + delta_i,
    for i = 0 .. len(scale) - 1. The coefficients carry the method; the loop
    is the same for all of them. Vectors keep the dtype of b (x0 is cast to
    it), so the same code evaluates the smoother in FP64 or in FP32.
    """
    if x_is_zero:
        x = np.zeros_like(b)
    else:
        x = np.array(x0, dtype=b.dtype, copy=True)
    delta = None
    for i, (cf, sf) in enumerate(zip(carry, scale)):
        res = b.copy() if (x_is_zero and i == 0) else b - apply_a(x)
        z = apply_m(res)
        delta = sf * z if delta is None else cf * delta + sf * z
        x = x + delta
    return x


def cheb4_coefficients(beta: float, k: int):
    """Increment coefficients of Algorithm 3 for degree k >= 1.

    Algorithm 3 moves x by (4 / beta) mu_i p_i with mu_i = (2i-1)/(2i+1)
    (mu_1 = 1/3 and mu_{i+1} = 1 / (2 - mu_i)) and p_i = mu_{i-1}^2 p_{i-1}
    + M r_{i-1}. For the increment delta_i = (4 / beta) mu_i p_i this gives
    delta_i = mu_i mu_{i-1} delta_{i-1} + (4 / beta) mu_i M r_{i-1}, where
    mu_i mu_{i-1} = (2i-3)/(2i+1).
    """
    if k < 1:
        raise ValueError("degree must be >= 1")
    mu = [(2 * i - 1) / (2 * i + 1) for i in range(1, k + 1)]
    scale = [4.0 * m / beta for m in mu]
    carry = [0.0] + [mu[i] * mu[i - 1] for i in range(1, k)]
    return carry, scale


def cheb4(apply_a, apply_m, b, x0, beta: float, k: int, x_is_zero: bool = False):
    """Algorithm 3: Chebyshev iteration of the fourth kind, degree k >= 1.

    apply_a(v) = A v, apply_m(v) = M v, beta >= lambda_max(MA).
    x_is_zero: x0 is zero, so the first residual is b itself.
    """
    carry, scale = cheb4_coefficients(beta, k)
    return _polynomial_smoother(apply_a, apply_m, b, x0, carry, scale, x_is_zero)


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


def cheb1_coefficients(alpha: float, beta: float, k: int):
    """Increment coefficients of Algorithm 2 on [alpha, beta], degree k >= 1.

    With c = (alpha + beta)/2 and d = (beta - alpha)/2, Algorithm 2 moves x by
    omega_i p_i, where omega_1 = 1/c, psi_1 = (d omega_1)^2 / 2,
    omega_{i+1} = 1 / (c - psi_i / omega_i), psi_{i+1} = (d omega_{i+1} / 2)^2
    and p_{i+1} = M r_i + psi_i p_i. The increment delta_i = omega_i p_i
    therefore obeys delta_{i+1} = (omega_{i+1} psi_i / omega_i) delta_i +
    omega_{i+1} M r_i.
    """
    if k < 1:
        raise ValueError("degree must be >= 1")
    if not 0 < alpha < beta:
        raise ValueError("need 0 < alpha < beta")
    c = 0.5 * (alpha + beta)
    d = 0.5 * (beta - alpha)
    omega = [1.0 / c]
    psi = [0.5 * (d * omega[0]) ** 2]
    for _ in range(1, k):
        omega.append(1.0 / (c - psi[-1] / omega[-1]))
        psi.append((d * omega[-1] / 2.0) ** 2)
    carry = [0.0] + [omega[i] * psi[i - 1] / omega[i - 1] for i in range(1, k)]
    return carry, omega


def cheb1(apply_a, apply_m, b, x0, alpha: float, beta: float, k: int, x_is_zero: bool = False):
    """Algorithm 2 (Chebyshev iteration of the first kind, degree k >= 1) with
    the preconditioner M applied to every residual, on [alpha, beta].

    As a smoother (Sec. 3.1) [alpha, beta] covers only the upper part of the
    spectrum of MA: alpha = rho lambda_max, rho in (0, 1)."""
    carry, scale = cheb1_coefficients(alpha, beta, k)
    return _polynomial_smoother(apply_a, apply_m, b, x0, carry, scale, x_is_zero)


def richardson(apply_a, apply_m, b, x0, omega: float, k: int, x_is_zero: bool = False):
    """Richardson smoothing: k steps x <- x + omega M (b - A x), i.e.
    S = (I - omega M A)^k (Sec. 3.1 takes omega = 1)."""
    if k < 1:
        raise ValueError("degree must be >= 1")
    return _polynomial_smoother(apply_a, apply_m, b, x0, [0.0] * k, [omega] * k, x_is_zero)


def t1_hat(k: int, lam, alpha: float, beta: float):
    """T^_k(lambda) = T_k((2 lambda - alpha - beta)/(beta - alpha)) /
    T_k((alpha + beta)/(alpha - beta)) (Eq. chebyshev_1st_kind), with T_k
    evaluated by numpy.polynomial.chebyshev (not by Algorithm 2's recurrence)."""
    from numpy.polynomial import chebyshev as npc
    coef = np.zeros(k + 1)
    coef[k] = 1.0
    lam = np.asarray(lam, dtype=np.float64)
    return npc.chebval((2.0 * lam - alpha - beta) / (beta - alpha), coef) / npc.chebval(
        (alpha + beta) / (alpha - beta), coef)


def poly_spectral(gmat: np.ndarray, amat: np.ndarray, b, x0, pfun):
    """x_k = x0 + G^T V diag((1 - p(lambda)) / lambda) V^T G r_0 for the
    residual polynomial p of the smoother (p(0) = 1), G A G^T = V Lambda V^T:
    the plain definition of any polynomial smoother with M = G^T G."""
    bmat = gmat @ amat @ gmat.T
    bmat = 0.5 * (bmat + bmat.T)
    lam, v = np.linalg.eigh(bmat)
    q = (1.0 - pfun(lam)) / lam
    r0 = b - amat @ x0
    return x0 + gmat.T @ (v @ (q * (v.T @ (gmat @ r0))))
