"""GPU parity of the hierarchy: Galerkin coarse operators, V(k,k) cycle and
FP64 PCG against the oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import multilevel, solver
from oracle.bsr import from_problem
from problems import make_problem, rhs
from tests.helpers import dev, gpu_levels, hierarchy_inputs, host, oracle_levels, rel_err, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def chf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2509_06744_amd as m
    m.lib()
    return m


def _oracle_levels(p, levels, mode="lower", tmax=0, seed=0):
    return oracle_levels(p, levels, mode, tmax, seed)


@pytest.mark.parametrize("n,b,levels", [(16, 3, 3), (32, 10, 3)])
def test_galerkin_operators(chf, n, b, levels):
    p = make_problem(n, 2, b, 2, seed=0)
    olv = _oracle_levels(p, levels)
    A, L, _, _ = gpu_levels(p, levels, 3, 0)
    for l in range(1, levels):
        Al, _, _ = chf.levels_get(L, l)
        rp, ci, vals = chf.bsr_export(Al)
        oa = olv[l].a
        assert np.array_equal(rp, oa.rowptr) and np.array_equal(ci, oa.colidx)
        assert rel_err(vals, oa.vals) < 1e-13


# b = 1 puts 64 block rows in a wavefront of the basis prolongation, b = 7 leaves
# one lane idle
@pytest.mark.parametrize("n,b,levels,degree", [(16, 3, 3, 2), (32, 10, 3, 3), (16, 1, 3, 2), (16, 7, 3, 2)])
def test_vcycle_matches_oracle(chf, n, b, levels, degree):
    import torch
    p = make_problem(n, 2, b, 2, seed=0)
    olv = _oracle_levels(p, levels)
    betas = [lv.beta for lv in olv[:-1]]
    A, L, _, _ = gpu_levels(p, levels, degree, 0, betas=betas)
    b_ = rhs(0, p.ndof)
    want = multilevel.vcycle(olv, 0, b_, degree)
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    chf.vcycle(L, dev(b_), x, x_is_zero=True)
    assert rel_err(host(x), want) < 1e-11
    # from a nonzero start
    x0 = np.random.default_rng(1).standard_normal(p.ndof)
    want2 = multilevel.vcycle_x(olv, b_, x0, degree)
    x = dev(x0)
    chf.vcycle(L, dev(b_), x, x_is_zero=False)
    assert rel_err(host(x), want2) < 1e-11


def test_lanczos_betas_per_level(chf):
    p = make_problem(32, 2, 10, 2, seed=0)
    olv = _oracle_levels(p, 3)
    A, L, _, _ = gpu_levels(p, 3, 3, 0)
    for l in range(2):
        assert abs(chf.levels_get_beta(L, l) - olv[l].beta) < 1e-9 * olv[l].beta


def test_pcg_config0(chf):
    """32x32 patches, b = 10, 3 levels, lower(A) pattern, degree 3, rtol 1e-8."""
    import torch
    p = make_problem(32, 2, 10, 2, seed=0)
    olv = _oracle_levels(p, 3)
    b_ = rhs(0, p.ndof)
    ox, oit, ohist, otrue = multilevel.pcg(olv[0].apply_a, lambda r: multilevel.vcycle(olv, 0, r, 3), b_, 1e-8, 100)
    A, L, _, _ = gpu_levels(p, 3, 3, 0)
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    it, hist, true_res, rc = chf.pcg_solve(L, dev(b_), x, rtol=1e-8, maxit=100)
    assert abs(it - oit) <= 1
    assert hist[-1] <= 1e-8 and true_res < 1e-7
    assert rel_err(host(x), ox) < 1e-6


def test_pcg_flexible_and_noconv(chf):
    import torch
    p = make_problem(16, 2, 3, 2, seed=2)
    A, L, _, _ = gpu_levels(p, 3, 2, 0, seed=2)
    b_ = dev(rhs(2, p.ndof))
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    it1, _, _, _ = chf.pcg_solve(L, b_, x, rtol=1e-8, maxit=100)
    it2, _, _, _ = chf.pcg_solve(L, b_, x, rtol=1e-8, maxit=100, flexible=True)
    assert abs(it1 - it2) <= 1
    it3, hist, _, rc = chf.pcg_solve(L, b_, x, rtol=1e-14, maxit=2, raise_on_noconv=False)
    assert rc == -5 and it3 == 2


def test_single_level_pcg_one_iteration(chf):
    import torch
    p = make_problem(6, 2, 3, 2, seed=0)
    A = chf.bsr_create(p.nb, p.b, p.rowptr, p.colidx, p.vals)
    L = chf.levels_create(A)
    chf.levels_setup(L, degree=2, pattern=0, v0=[])
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    it, hist, true_res, rc = chf.pcg_solve(L, dev(rhs(0, p.ndof)), x, rtol=1e-10, maxit=10)
    assert it == 1 and true_res < 1e-10


# Zero weights for coarse block 0 in the last prolongator make the coarsest
# Galerkin operator singular (its row 0 is zero), so its dense factorisation
# fails: CHF_ENOTSPD with bad_row -2. With 2 levels the coarsest level is
# factored on the calling thread, with 3 on the set-up's worker thread.
@pytest.mark.parametrize("levels", [2, 3])
def test_error_coarsest_not_spd_reports_minus_two(chf, levels):
    from problems import level_basis
    p = make_problem(16, 2, 3, 2, seed=0)
    A = upload(p)
    pro, starts = hierarchy_inputs(p.n, p.dim, p.b, levels, 0)
    L = chf.levels_create(A)
    for i, (ps, basis) in enumerate(zip(pro, level_basis(p, levels))):
        ps = ps.tocsr().copy()
        if i == levels - 2:
            ps.data[ps.indices == 0] = 0.0
        chf.levels_add_coarse(L, ps.shape[1], ps.indptr, ps.indices, ps.data, basis)
    with pytest.raises(chf.ChfError) as ei:
        chf.levels_setup(L, degree=2, pattern=0, v0=[dev(s) for s in starts[:-1]])
    assert ei.value.code == -3 and ei.value.bad_row == -2


def test_pcg_breakdown_keeps_last_iterate(chf):
    """Bounds beta_l ten times too small make the smoother's polynomial blow up
    on the upper spectrum, so the cycle is indefinite and r^T z < 0 at the
    first step (the oracle gives about -6e9 here): PCG reports CHF_EBREAKDOWN
    and leaves x at its start, zero."""
    import torch
    p = make_problem(16, 2, 3, 2, seed=2)
    A, L, _, _ = gpu_levels(p, 3, 2, 0, seed=2)
    for l in range(2):
        chf.levels_set_beta(L, l, 0.1 * chf.levels_get_beta(L, l))
    x = torch.full((p.ndof,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(chf.ChfError) as ei:
        chf.pcg_solve(L, dev(rhs(2, p.ndof)), x, rtol=1e-8, maxit=50)
    assert ei.value.code == -6
    assert not torch.any(x != 0)


def test_energy_factor_matches_oracle(chf):
    """chf_levels_energy_factor against the oracle's protocol (same bounds):
    a fixed number of cycles (tol 0), then to the tolerance."""
    from problems import uniform_start
    p = make_problem(16, 2, 3, 2, seed=0)
    olv = _oracle_levels(p, 3)
    betas = [lv.beta for lv in olv[:-1]]
    A, L, _, _ = gpu_levels(p, 3, 3, 0, betas=betas)
    e0 = uniform_start(0, p.ndof)
    for tol, maxit in [(0.0, 6), (1e-8, 50)]:
        want, wn = multilevel.energy_factor(olv, e0, 3, tol=tol, maxit=maxit)
        rho, n = chf.levels_energy_factor(L, dev(e0), tol=tol, maxit=maxit)
        assert n == wn
        assert abs(rho - want) < 1e-9 * want
