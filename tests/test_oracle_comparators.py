"""Pins for the oracle's comparator smoothers of Sec. 3.1 and the V(2k,0)
cycle of Sec. 5:

- Algorithm 2 (first-kind Chebyshev) against Eq. chebyshev_1st_kind evaluated
  with NumPy's Chebyshev series (not the algorithm's recurrence), on a
  diagonal operator and through the spectral definition with M = G^T G;
  its degree-1 closed form; the minimax value 1 / cosh(k arccosh((b+a)/(b-a)));
- Richardson smoothing against (I - omega M A)^k;
- V(2k,0) against its two-level error operator built from dense matrices,
  symmetry of V(k,k) for every smoother, and the lack of it for V(2k,0);
- BiCGStab (the outer solver for V(2k,0)) against a dense solve, and its
  one-step convergence with the exact preconditioner."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import chebyshev, fsai, multilevel, solver
from oracle.bsr import from_problem
from problems import grid_sizes, lanczos_starts, make_problem, prolongator


@pytest.mark.parametrize("k", range(1, 9))
def test_cheb1_diagonal_operator_closed_form(k):
    rng = np.random.default_rng(100 + k)
    n = 50
    lam = np.sort(rng.uniform(1e-3, 3.0, n))
    alpha, beta = 0.6, 3.0
    xstar = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    b = lam * xstar
    x = chebyshev.cheb1(lambda v: lam * v, lambda v: v, b, x0, alpha, beta, k)
    want = chebyshev.t1_hat(k, lam, alpha, beta) * (x0 - xstar)
    assert np.abs((x - xstar) - want).max() < 1e-12 * np.abs(x0 - xstar).max()


@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_cheb1_minimax_value(k):
    alpha, beta = 0.25, 2.0
    lam = np.linspace(alpha, beta, 200001)
    val = np.abs(chebyshev.t1_hat(k, lam, alpha, beta)).max()
    want = 1.0 / np.cosh(k * np.arccosh((beta + alpha) / (beta - alpha)))
    assert abs(val - want) < 1e-10
    assert abs(chebyshev.t1_hat(k, 0.0, alpha, beta) - 1.0) < 1e-14


@pytest.fixture(scope="module")
def small_system():
    p = make_problem(4, 2, 3, 2, seed=0)
    a = from_problem(p)
    g = fsai.fsai(a, *fsai.pattern_lower(a))
    ad, gd = a.dense(), g.dense()
    lmax = np.linalg.eigvalsh(gd @ ad @ gd.T).max()
    return ad, gd, lmax


@pytest.mark.parametrize("k", [1, 2, 3, 5])
def test_cheb1_matches_spectral_definition(small_system, k):
    ad, gd, lmax = small_system
    rng = np.random.default_rng(30 + k)
    b = rng.standard_normal(ad.shape[0])
    x0 = rng.standard_normal(ad.shape[0])
    beta = 1.01 * lmax
    alpha = 0.3 * beta
    m = gd.T @ gd
    x = chebyshev.cheb1(lambda v: ad @ v, lambda v: m @ v, b, x0, alpha, beta, k)
    xs = chebyshev.poly_spectral(gd, ad, b, x0, lambda t: chebyshev.t1_hat(k, t, alpha, beta))
    assert np.abs(x - xs).max() < 1e-10 * np.abs(xs).max()


def test_cheb1_degree_one(small_system):
    ad, gd, lmax = small_system
    rng = np.random.default_rng(5)
    b, x0 = rng.standard_normal((2, ad.shape[0]))
    m = gd.T @ gd
    x = chebyshev.cheb1(lambda v: ad @ v, lambda v: m @ v, b, x0, 1.0, 3.0, 1)
    assert np.allclose(x, x0 + 0.5 * (m @ (b - ad @ x0)), rtol=0, atol=1e-14 * np.abs(x).max())


@pytest.mark.parametrize("k,omega", [(1, 1.0), (3, 1.0), (4, 0.7), (6, 0.4)])
def test_richardson_error_operator(small_system, k, omega):
    ad, gd, lmax = small_system
    rng = np.random.default_rng(40 + k)
    b, x0 = rng.standard_normal((2, ad.shape[0]))
    m = gd.T @ gd
    x = chebyshev.richardson(lambda v: ad @ v, lambda v: m @ v, b, x0, omega, k)
    xstar = np.linalg.solve(ad, b)
    e = np.linalg.matrix_power(np.eye(ad.shape[0]) - omega * m @ ad, k) @ (x0 - xstar)
    assert np.abs((x - xstar) - e).max() < 1e-9 * np.abs(x0 - xstar).max()
    xs = chebyshev.poly_spectral(gd, ad, b, x0, lambda t: (1.0 - omega * t) ** k)
    assert np.abs(x - xs).max() < 1e-9 * np.abs(xs).max()


@pytest.mark.parametrize("smoother,param", [("cheb1", 0.3), ("richardson", 1.0)])
def test_zero_start_flag(small_system, smoother, param):
    ad, gd, lmax = small_system
    b = np.random.default_rng(3).standard_normal(ad.shape[0])
    m = gd.T @ gd
    if smoother == "cheb1":
        f = lambda x0, z: chebyshev.cheb1(lambda v: ad @ v, lambda v: m @ v, b, x0, param * lmax, lmax, 4,  # noqa: E731
                                          x_is_zero=z)
    else:
        f = lambda x0, z: chebyshev.richardson(lambda v: ad @ v, lambda v: m @ v, b, x0, param, 4,  # noqa: E731
                                               x_is_zero=z)
    assert np.array_equal(f(np.zeros_like(b), False), f(None, True))


def _hier(n=8, b=3, levels=2, seed=0):
    p = make_problem(n, 2, b, 2, seed=seed)
    a = from_problem(p)
    sizes = grid_sizes(n, levels)
    pro = [prolongator(sizes[l + 1], 2) for l in range(levels - 1)]
    starts = lanczos_starts(seed, [s * s * b for s in sizes])
    return p, solver.build_levels(a, pro, starts, "lower")


@pytest.mark.parametrize("smoother,param", [("cheb4", 0.0), ("cheb1", 0.3), ("richardson", 0.8)])
def test_v2k0_two_level_error_operator(smoother, param):
    """Two levels, exact coarse solve: V(2k,0) x = S_2k(b) followed by the
    coarse correction, i.e. error operator (I - P A_c^{-1} P^T A) p_2k(MA)."""
    p, levels = _hier()
    k = 2
    lev = levels[0]
    ad = lev.a.dense()
    gd = lev.g.dense()
    pb = lev.pb.toarray()
    ac = pb.T @ ad @ pb
    rng = np.random.default_rng(7)
    b = rng.standard_normal(ad.shape[0])
    x = multilevel.vcycle(levels, 0, b, k, smoother, param, cycle="v2k0")
    if smoother == "cheb4":
        pfun = lambda t: chebyshev.w4_hat(2 * k, t, lev.beta)  # noqa: E731
    elif smoother == "cheb1":
        pfun = lambda t: chebyshev.t1_hat(2 * k, t, param * lev.beta, lev.beta)  # noqa: E731
    else:
        pfun = lambda t: (1.0 - param * t) ** (2 * k)  # noqa: E731
    xs = chebyshev.poly_spectral(gd, ad, b, np.zeros_like(b), pfun)
    xs = xs + pb @ sla.solve(ac, pb.T @ (b - ad @ xs), assume_a="pos")
    assert np.abs(x - xs).max() < 1e-9 * np.abs(xs).max()


@pytest.mark.parametrize("smoother,param", [("cheb1", 0.3), ("richardson", 0.8)])
def test_vkk_symmetric_for_every_smoother(smoother, param):
    p, levels = _hier(n=16, levels=3)
    rng = np.random.default_rng(11)
    b1, b2 = rng.standard_normal((2, p.ndof))
    v1 = multilevel.vcycle(levels, 0, b1, 3, smoother, param)
    v2 = multilevel.vcycle(levels, 0, b2, 3, smoother, param)
    assert abs(v1 @ b2 - b1 @ v2) < 1e-11 * abs(v1 @ b2)


def test_v2k0_not_symmetric():
    p, levels = _hier(n=16, levels=3)
    rng = np.random.default_rng(12)
    b1, b2 = rng.standard_normal((2, p.ndof))
    v1 = multilevel.vcycle(levels, 0, b1, 2, cycle="v2k0")
    v2 = multilevel.vcycle(levels, 0, b2, 2, cycle="v2k0")
    assert abs(v1 @ b2 - b1 @ v2) > 1e-6 * abs(v1 @ b2)


def test_bicgstab_matches_dense_solve_with_nonsymmetric_preconditioner():
    p, levels = _hier(n=16, levels=3)
    a0 = levels[0]
    b = np.random.default_rng(21).standard_normal(p.ndof)
    x, it, hist, tr = multilevel.bicgstab(a0.apply_a, lambda r: multilevel.vcycle(levels, 0, r, 2, cycle="v2k0"),
                                          b, 1e-10, 200)
    xs = np.linalg.solve(a0.a.dense(), b)
    assert tr < 1e-9 and hist[-1] <= 1e-10
    assert np.abs(x - xs).max() < 1e-7 * np.abs(xs).max()
    assert it < 60


def test_bicgstab_exact_preconditioner_one_step():
    # with K = A^{-1} the first half step already solves the system
    p, levels = _hier(n=8, levels=2)
    ad = levels[0].a.dense()
    b = np.random.default_rng(22).standard_normal(p.ndof)
    x, it, hist, tr = multilevel.bicgstab(lambda v: ad @ v, lambda r: np.linalg.solve(ad, r), b, 1e-12, 10)
    assert it == 1 and len(hist) == 2 and tr < 1e-12
