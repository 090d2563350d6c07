"""Pins for the oracle's hierarchy: Galerkin variational identity, Lanczos
bounds, V(k,k) symmetry, exact one-level cycle, PCG against a dense solve,
scale invariance and a convergent energy-norm factor."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fsai, lanczos, multilevel, solver
from oracle.bsr import from_problem
from problems import grid_sizes, lanczos_starts, make_problem, prolongator, rhs


def _hier(n=16, b=3, levels=3, mode="lower", tmax=0, seed=0, scale=1.0, betas=None):
    p = make_problem(n, 2, b, 2, seed=seed)
    a = from_problem(p)
    a.vals = a.vals * scale
    sizes = grid_sizes(n, levels)
    pro = [prolongator(sizes[l + 1], 2) for l in range(levels - 1)]
    starts = lanczos_starts(seed, [s * s * b for s in sizes])
    return p, solver.build_levels(a, pro, starts, mode, tmax, betas=betas)


def test_galerkin_variational_identity():
    p = make_problem(16, 2, 3, 2, seed=1)
    a = from_problem(p)
    ps = prolongator(8, 2)
    ac = multilevel.galerkin(a, ps)
    pb = np.kron(ps.toarray(), np.eye(3))
    rng = np.random.default_rng(0)
    xc, yc = rng.standard_normal((2, ac.nb * 3))
    lhs = xc @ (ac.scipy() @ yc)
    rhs_ = (pb @ xc) @ (a.scipy() @ (pb @ yc))
    assert abs(lhs - rhs_) < 1e-12 * abs(rhs_)
    # coarse block stencil: 5x5 box in the interior
    assert max(np.diff(ac.rowptr)) == 25
    acd = ac.dense()
    assert abs(acd - acd.T).max() < 1e-13 * abs(acd).max()


def test_lanczos_brackets_lambda_max():
    p = make_problem(8, 2, 3, 2, seed=0)
    a = from_problem(p)
    g = fsai.fsai(a, *fsai.pattern_lower(a))
    gd, ad = g.dense(), a.dense()
    bm = gd @ ad @ gd.T
    lmax = np.linalg.eigvalsh(bm).max()
    v0 = lanczos_starts(0, [ad.shape[0]])[0]
    beta, theta = lanczos.lmax(lambda v: bm @ v, v0, 100, 1.01)
    assert theta <= lmax * (1 + 1e-12)
    assert beta >= lmax
    assert theta > 0.999 * lmax


def test_lanczos_small_invariant_subspace():
    # operator with 3 distinct eigenvalues: the recurrence stops early and the
    # Ritz value is exact
    d = np.array([1.0, 2.0, 5.0] * 10)
    v0 = np.ones(30)
    beta, theta = lanczos.lmax(lambda v: d * v, v0, 100, 1.0)
    assert abs(theta - 5.0) < 1e-12


def test_vcycle_symmetric():
    p, levels = _hier()
    rng = np.random.default_rng(3)
    n = p.ndof
    b1, b2 = rng.standard_normal((2, n))
    v1 = multilevel.vcycle(levels, 0, b1, 3)
    v2 = multilevel.vcycle(levels, 0, b2, 3)
    assert abs(v1 @ b2 - b1 @ v2) < 1e-12 * abs(v1 @ b2)
    # positive definite on random vectors
    assert v1 @ b1 > 0 and v2 @ b2 > 0


def test_single_level_is_exact_and_pcg_takes_one_step():
    p = make_problem(6, 2, 3, 2, seed=0)
    a = from_problem(p)
    levels = solver.build_levels(a, [], [], "lower")
    b = rhs(0, p.ndof)
    x, it, hist, true_res = multilevel.pcg(levels[0].apply_a, lambda r: multilevel.vcycle(levels, 0, r, 2),
                                           b, 1e-10, 10)
    assert it == 1 and true_res < 1e-10


def test_pcg_matches_dense_solve():
    p, levels = _hier(n=16, b=3, levels=3)
    b = rhs(0, p.ndof)
    x, it, hist, true_res = multilevel.pcg(levels[0].apply_a, lambda r: multilevel.vcycle(levels, 0, r, 3),
                                           b, 1e-10, 100)
    xd = sla.solve(levels[0].a.dense(), b, assume_a="pos")
    assert hist[-1] <= 1e-10
    assert np.linalg.norm(x - xd) <= 1e-6 * np.linalg.norm(xd)
    assert it < 40


def test_pcg_scale_invariance():
    # A -> alpha A leaves M A, beta and the iteration count unchanged
    p, l1 = _hier(n=16, b=3, levels=3)
    _, l2 = _hier(n=16, b=3, levels=3, scale=1000.0)
    b = rhs(0, p.ndof)
    r1 = multilevel.pcg(l1[0].apply_a, lambda r: multilevel.vcycle(l1, 0, r, 3), b, 1e-8, 100)
    r2 = multilevel.pcg(l2[0].apply_a, lambda r: multilevel.vcycle(l2, 0, r, 3), b, 1e-8, 100)
    assert r1[1] == r2[1]
    assert abs(l2[0].beta - l1[0].beta) < 1e-8 * l1[0].beta


def test_energy_factor_converges():
    from problems import uniform_start
    p, levels = _hier(n=16, b=3, levels=3)
    rho, n = multilevel.energy_factor(levels, uniform_start(0, p.ndof), 3)
    assert 0 < rho < 0.9


@pytest.mark.parametrize("ncyc", [1, 4, 9])
def test_energy_factor_against_dense_error_operator(ncyc):
    # Two levels with an exact coarse solve: the cycle on b = 0 maps e to
    # E e, E = p(MA) (I - P A_c^{-1} P^T A) p(MA), p = W^_k on [0, beta], with
    # p(MA) formed from the eigendecomposition of G A G^T. The factor after n
    # cycles is (||E^n e0||_A / ||e0||_A)^{1/n}.
    from oracle import chebyshev
    from problems import uniform_start
    p, levels = _hier(n=8, b=3, levels=2)
    k = 3
    lev = levels[0]
    ad, gd, pb = lev.a.dense(), lev.g.dense(), lev.pb.toarray()
    bmat = gd @ ad @ gd.T
    lam, v = np.linalg.eigh(0.5 * (bmat + bmat.T))
    q = (1.0 - chebyshev.w4_hat(k, lam, lev.beta)) / lam
    smooth = np.eye(ad.shape[0]) - gd.T @ (v * q) @ v.T @ gd @ ad
    coarse = np.eye(ad.shape[0]) - pb @ np.linalg.solve(pb.T @ ad @ pb, pb.T @ ad)
    err = smooth @ coarse @ smooth
    e0 = uniform_start(3, p.ndof)
    en = np.linalg.matrix_power(err, ncyc) @ e0
    want = np.sqrt((en @ ad @ en) / (e0 @ ad @ e0)) ** (1.0 / ncyc)
    rho, n = multilevel.energy_factor(levels, e0, k, tol=0.0, maxit=ncyc)
    assert n == ncyc
    assert abs(rho - want) < 1e-10 * want


def test_pcg_flexible_variant_close():
    p, levels = _hier(n=16, b=3, levels=3)
    b = rhs(1, p.ndof)
    r1 = multilevel.pcg(levels[0].apply_a, lambda r: multilevel.vcycle(levels, 0, r, 3), b, 1e-8, 100)
    r2 = multilevel.pcg(levels[0].apply_a, lambda r: multilevel.vcycle(levels, 0, r, 3), b, 1e-8, 100,
                        flexible=True)
    assert abs(r1[1] - r2[1]) <= 1


def test_basis_transfer_reduces_to_scalar_galerkin():
    # With P = R^{-1} (P_s (x) I_b), T^T A T = D (x) I_b, so the coarse operator
    # is the scalar Galerkin product of D repeated per block component.
    import scipy.sparse as sp
    from problems import level_basis
    p = make_problem(16, 2, 3, 2, seed=5)
    a = from_problem(p)
    ps = prolongator(8, 2)
    ac = multilevel.galerkin(a, ps, level_basis(p, 2)[0]).dense()
    dc = (ps.T @ p.dstencil @ ps).toarray()
    want = np.kron(dc, np.eye(3))
    assert abs(ac - want).max() < 1e-12 * abs(want).max()


def test_basis_transfer_pcg_iterations_bounded():
    from tests.helpers import oracle_levels
    its = []
    for n in (16, 32):
        p = make_problem(n, 2, 10, 2, seed=0)
        lv = oracle_levels(p, 3)
        _, it, _, _ = multilevel.pcg(lv[0].apply_a, lambda r: multilevel.vcycle(lv, 0, r, 3), rhs(0, p.ndof), 1e-8, 200)
        its.append(it)
    assert its[1] <= 15 and its[1] <= its[0] + 6


def test_lanczos_reproduces_a_tridiagonal_operator():
    # Started from e_1, the Lanczos recurrence on a symmetric tridiagonal
    # matrix rebuilds that matrix (up to the signs of the basis vectors): for
    # tridiag(-1, 2, -1) every alpha is 2 and every beta is 1, exactly, and
    # the Ritz value after n steps is the largest eigenvalue 2 + 2 cos(pi/(n+1)).
    n = 24
    main = np.full(n, 2.0)
    off = np.full(n - 1, -1.0)

    def apply(v):
        w = main * v
        w[:-1] += off * v[1:]
        w[1:] += off * v[:-1]
        return w

    v0 = np.zeros(n)
    v0[0] = 1.0
    alphas, betas = lanczos.lanczos_tridiag(apply, v0, n)
    assert np.array_equal(alphas, np.full(n, 2.0))
    assert np.array_equal(betas, np.full(n - 1, 1.0))
    _, theta = lanczos.lmax(apply, v0, n, 1.0)
    assert abs(theta - (2.0 + 2.0 * np.cos(np.pi / (n + 1)))) < 1e-13
    # fewer steps: the Ritz value is the largest eigenvalue of the leading
    # m x m block, 2 + 2 cos(pi/(m+1))
    m = 7
    _, theta_m = lanczos.lmax(apply, v0, m, 1.0)
    assert abs(theta_m - (2.0 + 2.0 * np.cos(np.pi / (m + 1)))) < 1e-13


def test_lanczos_ritz_values_of_the_krylov_space():
    # After m steps the tridiagonal is the operator compressed to the Krylov
    # space K_m(B, v0): its eigenvalues equal those of Q^T B Q for any
    # orthonormal basis Q of that space (here from a QR of the Krylov matrix).
    rng = np.random.default_rng(5)
    n, m = 40, 6
    qf, _ = np.linalg.qr(rng.standard_normal((n, n)))
    bm = qf @ np.diag(np.linspace(1.0, 3.0, n)) @ qf.T
    v0 = rng.standard_normal(n)
    alphas, betas = lanczos.lanczos_tridiag(lambda v: bm @ v, v0, m)
    kry = np.empty((n, m))
    kry[:, 0] = v0 / np.linalg.norm(v0)
    for j in range(1, m):
        kry[:, j] = bm @ kry[:, j - 1]
    q, _ = np.linalg.qr(kry)
    want = np.linalg.eigvalsh(q.T @ bm @ q)
    t = np.diag(alphas) + np.diag(betas, 1) + np.diag(betas, -1)
    got = np.linalg.eigvalsh(t)
    assert np.abs(got - want).max() < 1e-10
    # the first Ritz value is the Rayleigh quotient of the start vector
    v = v0 / np.linalg.norm(v0)
    assert abs(alphas[0] - v @ bm @ v) < 1e-14 * abs(alphas[0])
