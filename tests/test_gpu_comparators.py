"""GPU parity of the comparator smoothers of Sec. 3.1 (first-kind Chebyshev,
Algorithm 2; Richardson smoothing), of the V(2k,0) cycle of Sec. 5 and of
BiCGStab, its outer solver, against the oracle, through the C ABI; error
paths of the new entry points."""
import numpy as np
import pytest

from oracle import chebyshev, fsai, lanczos, multilevel
from oracle.bsr import from_problem
from problems import lanczos_starts, make_problem, rhs
from tests.helpers import dev, gpu_levels, host, oracle_levels, rel_err, upload

pytestmark = pytest.mark.gpu

CASES = [(7, 2, 3, 2), (13, 2, 10, 2), (9, 2, 21, 3), (5, 3, 10, 2), (32, 2, 10, 2)]


@pytest.fixture(scope="module")
def chf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2509_06744_amd as m
    m.lib()
    return m


def _setup(chf, n, dim, b, pw):
    p = make_problem(n, dim, b, pw, seed=0)
    a = from_problem(p)
    og = fsai.fsai(a, *fsai.pattern_lower(a))
    asp, gsp = a.scipy(), og.scipy()
    gtsp = gsp.T.tocsr()
    beta, _ = lanczos.lmax(lambda v: gsp @ (asp @ (gtsp @ v)), lanczos_starts(0, [p.ndof])[0])
    A = upload(p)
    G = chf.fsai_setup(A, chf.pattern_lower(A))
    return p, asp, gsp, gtsp, beta, A, G


@pytest.mark.parametrize("n,dim,b,pw", CASES)
@pytest.mark.parametrize("degree", [1, 3, 4])
@pytest.mark.parametrize("x_is_zero", [False, True])
def test_cheb1_smoother(chf, n, dim, b, pw, degree, x_is_zero):
    import torch
    p, asp, gsp, gtsp, beta, A, G = _setup(chf, n, dim, b, pw)
    alpha = 0.3 * beta
    rng = np.random.default_rng(degree)
    b_ = rhs(0, p.ndof)
    x0 = np.zeros(p.ndof) if x_is_zero else rng.standard_normal(p.ndof)
    want = chebyshev.cheb1(lambda v: asp @ v, lambda v: gtsp @ (gsp @ v), b_, x0, alpha, beta, degree,
                           x_is_zero=x_is_zero)
    x = dev(x0 if not x_is_zero else np.full(p.ndof, np.nan))
    work = torch.empty(3 * p.ndof, dtype=torch.float64, device="cuda")
    chf.cheb1_smooth(A, G, alpha, beta, degree, dev(b_), x, x_is_zero=x_is_zero, work=work)
    assert rel_err(host(x), want) < 1e-12


@pytest.mark.parametrize("n,dim,b,pw", CASES)
@pytest.mark.parametrize("degree,omega", [(1, 1.0), (3, 1.0), (4, 0.6)])
@pytest.mark.parametrize("x_is_zero", [False, True])
def test_richardson_smoother(chf, n, dim, b, pw, degree, omega, x_is_zero):
    import torch
    p, asp, gsp, gtsp, beta, A, G = _setup(chf, n, dim, b, pw)
    rng = np.random.default_rng(degree)
    b_ = rhs(0, p.ndof)
    x0 = np.zeros(p.ndof) if x_is_zero else rng.standard_normal(p.ndof)
    want = chebyshev.richardson(lambda v: asp @ v, lambda v: gtsp @ (gsp @ v), b_, x0, omega, degree,
                                x_is_zero=x_is_zero)
    x = dev(x0 if not x_is_zero else np.full(p.ndof, np.nan))
    work = torch.empty(3 * p.ndof, dtype=torch.float64, device="cuda")
    chf.richardson_smooth(A, G, omega, degree, dev(b_), x, x_is_zero=x_is_zero, work=work)
    assert rel_err(host(x), want) < 1e-12


def test_comparator_errors(chf):
    import torch
    p, asp, gsp, gtsp, beta, A, G = _setup(chf, 5, 2, 3, 2)
    z = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    w = torch.zeros(3 * p.ndof, dtype=torch.float64, device="cuda")
    for alpha, bt, k in [(1.0, 1.0, 2), (-0.1, 1.0, 2), (0.2, 1.0, 0)]:
        with pytest.raises(chf.ChfError) as ei:
            chf.cheb1_smooth(A, G, alpha, bt, k, z, z, work=w)
        assert ei.value.code == -1
    for om, k in [(0.0, 2), (-1.0, 2), (1.0, 0)]:
        with pytest.raises(chf.ChfError) as ei:
            chf.richardson_smooth(A, G, om, k, z, z, work=w)
        assert ei.value.code == -1


CYCLES = [("cheb4", 0.0, "vkk"), ("cheb1", 0.3, "vkk"), ("richardson", 0.8, "vkk"),
          ("cheb4", 0.0, "v2k0"), ("cheb1", 0.3, "v2k0"), ("richardson", 1.0, "v2k0")]


def _code(chf, smoother, cycle):
    sm = {"cheb4": chf.SMOOTH_CHEB4, "cheb1": chf.SMOOTH_CHEB1, "richardson": chf.SMOOTH_RICHARDSON}[smoother]
    return sm, chf.CYCLE_V2K0 if cycle == "v2k0" else chf.CYCLE_VKK


@pytest.mark.parametrize("smoother,param,cycle", CYCLES)
@pytest.mark.parametrize("n,b,levels,degree", [(16, 3, 3, 2), (32, 10, 3, 3)])
def test_cycle_matches_oracle(chf, smoother, param, cycle, n, b, levels, degree):
    import torch
    p = make_problem(n, 2, b, 2, seed=0)
    olv = oracle_levels(p, levels)
    betas = [lv.beta for lv in olv[:-1]]
    A, L, _, _ = gpu_levels(p, levels, degree, 0, betas=betas)
    sm, cy = _code(chf, smoother, cycle)
    chf.levels_set_cycle(L, sm, param, cy)
    b_ = rhs(0, p.ndof)
    want = multilevel.vcycle(olv, 0, b_, degree, smoother, param, cycle)
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    chf.vcycle(L, dev(b_), x, x_is_zero=True)
    assert rel_err(host(x), want) < 1e-11
    x0 = np.random.default_rng(1).standard_normal(p.ndof)
    want2 = multilevel.vcycle_x(olv, b_, x0, degree, smoother, param, cycle)
    x = dev(x0)
    chf.vcycle(L, dev(b_), x, x_is_zero=False)
    assert rel_err(host(x), want2) < 1e-11


def test_v2k0_pcg_needs_flexible_and_matches_oracle(chf):
    """32x32 patches, b = 10, 3 levels, degree 2: V(4,0) with flexible CG."""
    import torch
    p = make_problem(32, 2, 10, 2, seed=0)
    olv = oracle_levels(p, 3)
    b_ = rhs(0, p.ndof)
    ox, oit, _, _ = multilevel.pcg(olv[0].apply_a, lambda r: multilevel.vcycle(olv, 0, r, 2, cycle="v2k0"), b_,
                                   1e-8, 100, flexible=True)
    A, L, _, _ = gpu_levels(p, 3, 2, 0)
    chf.levels_set_cycle(L, chf.SMOOTH_CHEB4, 0.0, chf.CYCLE_V2K0)
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    with pytest.raises(chf.ChfError) as ei:
        chf.pcg_solve(L, dev(b_), x, rtol=1e-8, maxit=100)
    assert ei.value.code == -1
    it, hist, true_res, rc = chf.pcg_solve(L, dev(b_), x, rtol=1e-8, maxit=100, flexible=True)
    assert abs(it - oit) <= 1
    assert hist[-1] <= 1e-8 and true_res < 1e-7
    assert rel_err(host(x), ox) < 1e-6


def test_set_cycle_errors(chf):
    p = make_problem(8, 2, 3, 2, seed=0)
    A, L, _, _ = gpu_levels(p, 2, 2, 0)
    for sm, par, cy in [(3, 0.0, 0), (0, 0.0, 2), (1, 0.0, 0), (1, 1.0, 0), (2, 0.0, 0), (2, -1.0, 0)]:
        with pytest.raises(chf.ChfError) as ei:
            chf.levels_set_cycle(L, sm, par, cy)
        assert ei.value.code == -1


@pytest.mark.parametrize("cycle", ["v2k0", "vkk"])
def test_bicgstab_matches_oracle(chf, cycle):
    """32x32 patches, b = 10, 3 levels, degree 2, BiCGStab to 1e-8."""
    import torch
    p = make_problem(32, 2, 10, 2, seed=0)
    olv = oracle_levels(p, 3)
    b_ = rhs(0, p.ndof)
    ox, oit, ohist, _ = multilevel.bicgstab(olv[0].apply_a, lambda r: multilevel.vcycle(olv, 0, r, 2, cycle=cycle),
                                            b_, 1e-8, 100)
    A, L, _, _ = gpu_levels(p, 3, 2, 0)
    chf.levels_set_cycle(L, chf.SMOOTH_CHEB4, 0.0, chf.CYCLE_V2K0 if cycle == "v2k0" else chf.CYCLE_VKK)
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    it, hist, true_res, rc = chf.bicgstab_solve(L, dev(b_), x, rtol=1e-8, maxit=100)
    assert abs(it - oit) <= 1
    assert hist[-1] <= 1e-8 and true_res < 1e-7
    m = min(len(hist), len(ohist), 6)
    assert np.allclose(hist[:m], ohist[:m], rtol=1e-6)
    assert rel_err(host(x), ox) < 1e-6


def test_bicgstab_zero_rhs_and_errors(chf):
    import torch
    p = make_problem(8, 2, 3, 2, seed=0)
    A, L, _, _ = gpu_levels(p, 2, 2, 0)
    z = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    x = torch.ones(p.ndof, dtype=torch.float64, device="cuda")
    it, hist, tr, rc = chf.bicgstab_solve(L, z, x, rtol=1e-8, maxit=10)
    assert it == 0 and rc == 0 and float(x.abs().max()) == 0.0
    with pytest.raises(chf.ChfError) as ei:
        chf.bicgstab_solve(L, z, x, rtol=-1.0, maxit=10)
    assert ei.value.code == -1
