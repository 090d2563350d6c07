"""Pins for the oracle's Algorithm 3 (fourth-kind Chebyshev smoothing):
closed-form error polynomial on a diagonal operator, the spectral plain
definition, the increment form, the smoothing bound of Lemma 3.2 and the
value W_k(1) = 2k+1."""
import numpy as np
import pytest

from oracle import chebyshev, fsai
from oracle.bsr import from_problem
from problems import make_problem


def _w4_closed(k, lam, beta):
    # W_k(cos t) = sin((k + 1/2) t) / sin(t / 2), normalised by W_k(1) = 2k + 1
    t = np.arccos(np.clip(1.0 - 2.0 * lam / beta, -1, 1))
    return np.sin((k + 0.5) * t) / ((2 * k + 1) * np.sin(t / 2))


@pytest.mark.parametrize("k", range(1, 11))
def test_diagonal_operator_closed_form(k):
    rng = np.random.default_rng(k)
    n = 60
    lam = np.sort(rng.uniform(1e-3, 2.0, n))
    beta = 2.0
    xstar = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    b = lam * xstar
    x = chebyshev.cheb4(lambda v: lam * v, lambda v: v, b, x0, beta, k)
    want = _w4_closed(k, lam, beta) * (x0 - xstar)
    assert np.abs((x - xstar) - want).max() < 1e-13 * np.abs(x0 - xstar).max()


@pytest.mark.parametrize("k", [1, 2, 5, 9])
def test_w4_value_at_one_and_recurrence(k):
    assert chebyshev.w4(k, 1.0) == 2 * k + 1
    assert abs(chebyshev.w4_hat(k, 0.0, 3.0) - 1.0) < 1e-15
    t = np.linspace(-0.99, 0.99, 37)
    assert np.allclose(chebyshev.w4(k, t), np.sin((k + 0.5) * np.arccos(t)) / np.sin(np.arccos(t) / 2))


@pytest.mark.parametrize("k", [1, 2, 3, 4, 6, 10])
def test_smoothing_bound(k):
    # max over [0, beta] of sqrt(lambda) |W^_k(lambda)| equals sqrt(beta)/(2k+1)
    beta = 5.0
    lam = np.linspace(0, beta, 400001)
    val = np.sqrt(lam) * np.abs(chebyshev.w4_hat(k, lam, beta))
    assert abs(val.max() - np.sqrt(beta) / (2 * k + 1)) < 1e-6 * np.sqrt(beta)
    # the alternation points of Lemma 3.2, theta_i = 2 i pi / (2k+1), attain it
    th = 2 * np.arange(k + 1) * np.pi / (2 * k + 1)
    lam_i = beta * (1 + np.cos(th)) / 2     # t_i = cos(theta_i) mapped by t = -(1 - 2 lam/beta)
    vals = np.sqrt(lam_i[1:]) * np.abs(chebyshev.w4_hat(k, lam_i[1:], beta))
    assert np.allclose(vals, np.sqrt(beta) / (2 * k + 1), rtol=1e-12)


@pytest.mark.parametrize("k", [2, 3, 5])
def test_weighted_minimax_optimality(k):
    # Random admissible perturbations (p(0) = 1 kept) never lower the weighted max.
    beta = 1.0
    lam = np.linspace(0, beta, 20001)
    best = (np.sqrt(lam) * np.abs(chebyshev.w4_hat(k, lam, beta))).max()
    rng = np.random.default_rng(k)
    for _ in range(50):
        coef = rng.standard_normal(k) * 1e-2
        pert = sum(c * lam ** (i + 1) for i, c in enumerate(coef))
        val = (np.sqrt(lam) * np.abs(chebyshev.w4_hat(k, lam, beta) + pert)).max()
        assert val >= best * (1 - 1e-12)


@pytest.fixture(scope="module")
def small_system():
    p = make_problem(4, 2, 3, 2, seed=0)
    a = from_problem(p)
    g = fsai.fsai(a, *fsai.pattern_lower(a))
    ad, gd = a.dense(), g.dense()
    lmax = np.linalg.eigvalsh(gd @ ad @ gd.T).max()
    return ad, gd, lmax


@pytest.mark.parametrize("k", [1, 2, 3, 4, 7])
def test_matches_spectral_definition(small_system, k):
    ad, gd, lmax = small_system
    rng = np.random.default_rng(10 + k)
    b = rng.standard_normal(ad.shape[0])
    x0 = rng.standard_normal(ad.shape[0])
    beta = 1.01 * lmax
    m = gd.T @ gd
    x = chebyshev.cheb4(lambda v: ad @ v, lambda v: m @ v, b, x0, beta, k)
    xs = chebyshev.cheb4_spectral(gd, ad, b, x0, beta, k)
    assert np.abs(x - xs).max() < 1e-10 * np.abs(xs).max()


@pytest.mark.parametrize("k", [1, 2, 3, 4, 8])
def test_matches_increment_form(small_system, k):
    ad, gd, lmax = small_system
    rng = np.random.default_rng(20 + k)
    b = rng.standard_normal(ad.shape[0])
    x0 = rng.standard_normal(ad.shape[0])
    m = gd.T @ gd
    x1 = chebyshev.cheb4(lambda v: ad @ v, lambda v: m @ v, b, x0, lmax, k)
    x2 = chebyshev.cheb4_increment_form(lambda v: ad @ v, lambda v: m @ v, b, x0, lmax, k)
    assert np.abs(x1 - x2).max() <= 1e-14 * np.abs(x1).max() * 10


def test_zero_start_flag(small_system):
    ad, gd, lmax = small_system
    b = np.random.default_rng(3).standard_normal(ad.shape[0])
    m = gd.T @ gd
    x1 = chebyshev.cheb4(lambda v: ad @ v, lambda v: m @ v, b, np.zeros_like(b), lmax, 4)
    x2 = chebyshev.cheb4(lambda v: ad @ v, lambda v: m @ v, b, None, lmax, 4, x_is_zero=True)
    assert np.array_equal(x1, x2)
