"""GPU parity of nested block-FSAI (Sec. 2.2, one nesting level) against the
oracle, through the C ABI: the triple product G0 A G0^T (structure bit-exact,
values 1e-12), the inner pattern from Algorithm 1 (bit-exact), the inner
factor (1e-12), and the nested factor inside the smoother, Lanczos and the
plain application; error paths."""
import numpy as np
import pytest

from oracle import adaptive, chebyshev, fsai, lanczos, nested
from oracle.bsr import from_problem
from problems import lanczos_starts, make_problem, rhs
from tests.helpers import dev, host, rel_err, upload

pytestmark = pytest.mark.gpu

CASES = [(8, 2, 3, 2, 3), (13, 2, 10, 2, 4), (4, 3, 10, 2, 3), (6, 2, 21, 3, 2)]


@pytest.fixture(scope="module")
def chf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2509_06744_amd as m
    m.lib()
    return m


def _both(chf, n, dim, b, pw, tmax):
    p = make_problem(n, dim, b, pw, seed=0)
    a = from_problem(p)
    p0 = adaptive.adaptive_pattern(a, tmax)
    og0, oa1, op1, og1 = nested.nested(a, p0, tmax)
    A = upload(p)
    G0 = chf.fsai_setup(A, chf.pattern_from_csr(p.nb, *p0))
    A1 = chf.bsr_triple(A, G0)
    P1 = chf.pattern_adaptive(A1, tmax)
    G1 = chf.fsai_setup(A1, P1)
    return p, a, (og0, oa1, op1, og1), (A, G0, A1, P1, G1)


@pytest.mark.parametrize("n,dim,b,pw,tmax", CASES)
def test_triple_product_inner_pattern_and_factor(chf, n, dim, b, pw, tmax):
    p, a, (og0, oa1, op1, og1), (A, G0, A1, P1, G1) = _both(chf, n, dim, b, pw, tmax)
    rp, ci, vals = chf.bsr_export(A1)
    assert np.array_equal(rp, oa1.rowptr) and np.array_equal(ci, oa1.colidx)
    assert rel_err(vals, oa1.vals) < 1e-12
    prow, pcol = chf.pattern_export(P1)
    assert np.array_equal(prow, op1[0]) and np.array_equal(pcol, op1[1])
    g1 = chf.fsai_export(G1, len(pcol), b)
    assert rel_err(g1, og1.vals) < 1e-12


@pytest.mark.parametrize("n,dim,b,pw,tmax", CASES)
@pytest.mark.parametrize("x_is_zero", [False, True])
def test_nested_smoother_and_lanczos(chf, n, dim, b, pw, tmax, x_is_zero):
    import torch
    p, a, (og0, oa1, op1, og1), (A, G0, A1, P1, G1) = _both(chf, n, dim, b, pw, tmax)
    Gn = chf.fsai_nest(G0, G1)
    am = nested.apply_m(og0, og1)
    asp = a.scipy()
    gh0, gh1 = og0.scipy(), og1.scipy()
    v0 = lanczos_starts(0, [p.ndof])[0]
    # Lanczos on G^ A G^T with G^ = G1 G0
    want_beta, want_theta = lanczos.lmax(lambda v: gh1 @ (gh0 @ (asp @ (gh0.T @ (gh1.T @ v)))), v0)
    beta, theta = chf.lmax_lanczos(A, Gn, dev(v0))
    assert abs(theta - want_theta) < 1e-9 * want_theta
    # one fourth-kind application with the nested M
    k = 3
    rng = np.random.default_rng(5)
    b_ = rhs(0, p.ndof)
    x0 = np.zeros(p.ndof) if x_is_zero else rng.standard_normal(p.ndof)
    want = chebyshev.cheb4(lambda v: asp @ v, am, b_, x0, want_beta, k, x_is_zero=x_is_zero)
    x = dev(x0 if not x_is_zero else np.full(p.ndof, np.nan))
    work = torch.empty(3 * p.ndof, dtype=torch.float64, device="cuda")
    chf.cheb4_smooth(A, Gn, want_beta, k, dev(b_), x, x_is_zero=x_is_zero, work=work)
    assert rel_err(host(x), want) < 1e-12
    # z = M r
    r = rng.standard_normal(p.ndof)
    z = torch.empty(p.ndof, dtype=torch.float64, device="cuda")
    chf.fsai_apply(Gn, dev(r), z, torch.empty(p.ndof, dtype=torch.float64, device="cuda"))
    assert rel_err(host(z), am(r)) < 1e-12


def test_nested_errors(chf):
    p, a, _, (A, G0, A1, P1, G1) = _both(chf, 6, 2, 3, 2, 2)
    Gn = chf.fsai_nest(G0, G1)
    with pytest.raises(chf.ChfError) as ei:
        chf.fsai_export(Gn, 10, 3)
    assert ei.value.code == -1
    with pytest.raises(chf.ChfError) as ei:
        chf.bsr_triple(A, Gn)
    assert ei.value.code == -1
    with pytest.raises(chf.ChfError) as ei:
        chf.fsai_nest(Gn, G1)
    assert ei.value.code == -1
    q = make_problem(5, 2, 3, 2, seed=0)
    B = upload(q)
    Gq = chf.fsai_setup(B, chf.pattern_lower(B))
    with pytest.raises(chf.ChfError) as ei:
        chf.fsai_nest(G0, Gq)
    assert ei.value.code == -1


def test_nested_hierarchy_vcycle_and_pcg(chf):
    """16x16 patches, b = 10, 3 levels, adaptive t_max 3 with one nesting
    level: Lanczos bounds, one V(2,2) cycle and PCG against the oracle."""
    import torch
    import paper_2509_06744_amd as m
    from oracle import multilevel
    from problems import level_basis
    from tests.helpers import hierarchy_inputs, oracle_levels
    p = make_problem(16, 2, 10, 2, seed=0)
    olv = oracle_levels(p, 3, "adaptive", 3, nest=True)
    A = upload(p)
    pro, starts = hierarchy_inputs(p.n, p.dim, p.b, 3, 0)
    L = m.levels_create(A)
    for ps, basis in zip(pro, level_basis(p, 3)):
        ps = ps.tocsr()
        m.levels_add_coarse(L, ps.shape[1], ps.indptr, ps.indices, ps.data, basis)
    m.levels_set_nesting(L, 1)
    m.levels_setup(L, degree=2, pattern=1, tmax=3, v0=[dev(s) for s in starts[:-1]])
    for l in range(2):
        assert abs(m.levels_get_beta(L, l) - olv[l].beta) < 1e-9 * olv[l].beta
        m.levels_set_beta(L, l, olv[l].beta)
    b_ = rhs(0, p.ndof)
    want = multilevel.vcycle(olv, 0, b_, 2)
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    m.vcycle(L, dev(b_), x, x_is_zero=True)
    assert rel_err(host(x), want) < 1e-11
    _, oit, _, _ = multilevel.pcg(olv[0].apply_a, lambda r: multilevel.vcycle(olv, 0, r, 2), b_, 1e-8, 100)
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    it, hist, tr, rc = m.pcg_solve(L, dev(b_), x, rtol=1e-8, maxit=100)
    assert abs(it - oit) <= 1 and tr < 1e-7
    L2 = m.levels_create(A)
    with pytest.raises(m.ChfError):
        m.levels_set_nesting(L2, 2)
