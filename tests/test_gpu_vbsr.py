"""GPU parity for variable block sizes (Def. 2.1 with unequal m_i; Sec. 5
Ex. 5.1's degree bump on the boundary patches): the SpMV layout, the
block-FSAI set-up, the smoother and the Lanczos bound against the
variable-block oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import chebyshev, fsai, lanczos, vbsr
from problems import lanczos_starts, make_vb_problem, rhs
from tests.helpers import dev, host, rel_err

pytestmark = pytest.mark.gpu

# (patches per side, dimension, D = L^power, interior degree, boundary degree):
# 2D p = 2 / 3 (6 and 10 unknowns), 3D p = 1 / 2 (4 and 10), 2D p = 1 / 4
# (3 and 15: odd widths), and equal degrees (uniform sizes through this path)
CASES = [(9, 2, 2, 2, 3), (4, 3, 2, 1, 2), (7, 2, 3, 1, 4), (6, 2, 2, 2, 2)]


@pytest.fixture(scope="module")
def chf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2509_06744_amd as m
    m.lib()
    return m


def _upload(chf, p):
    return chf.vbsr_create(p.nb, p.bsize, p.rowptr, p.colidx, p.vals)


@pytest.mark.parametrize("n,dim,pw,pi,pb", CASES)
def test_vbsr_spmv_and_export(chf, n, dim, pw, pi, pb):
    import torch
    p = make_vb_problem(n, dim, pw, pi, pb, seed=1)
    a = vbsr.from_problem(p)
    A = _upload(chf, p)
    nd, nv, bs = chf.vbsr_info(A)
    assert nd == p.ndof and nv == len(p.vals) and np.array_equal(bs, p.bsize)
    x = np.random.default_rng(0).standard_normal(p.ndof)
    bv = np.random.default_rng(1).standard_normal(p.ndof)
    y = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    chf.bsr_spmv(A, dev(x), y)
    asp = a.scipy()
    assert rel_err(host(y), asp @ x) < 1e-13
    chf.bsr_spmv(A, dev(x), y, bvec=dev(bv))
    assert rel_err(host(y), bv - asp @ x) < 1e-13
    with pytest.raises(chf.ChfError):
        chf.bsr_spmv(A, dev(x).float(), y.float(), dtype=chf.F32)


@pytest.mark.parametrize("n,dim,pw,pi,pb", CASES)
def test_vbsr_fsai_lower_pattern(chf, n, dim, pw, pi, pb):
    p = make_vb_problem(n, dim, pw, pi, pb, seed=2)
    a = vbsr.from_problem(p)
    prow, pcol = fsai.pattern_lower(a)
    og = vbsr.fsai(a, prow, pcol)
    A = _upload(chf, p)
    P = chf.pattern_lower(A)
    r2, c2 = chf.pattern_export(P)
    assert np.array_equal(r2, prow) and np.array_equal(c2, pcol)
    G = chf.fsai_setup(A, P)
    g = chf.fsai_export_flat(G, len(og.vals))
    assert rel_err(g, og.vals) < 1e-12


@pytest.mark.parametrize("n,dim,pw,pi,pb", CASES[:3])
@pytest.mark.parametrize("degree,x_is_zero", [(1, True), (4, False), (3, True)])
def test_vbsr_smoother_and_lanczos(chf, n, dim, pw, pi, pb, degree, x_is_zero):
    import torch
    p = make_vb_problem(n, dim, pw, pi, pb, seed=3)
    a = vbsr.from_problem(p)
    prow, pcol = fsai.pattern_lower(a)
    gsp = vbsr.fsai(a, prow, pcol).scipy()
    gtsp = gsp.T.tocsr()
    asp = a.scipy()
    v0 = lanczos_starts(3, [p.ndof])[0]
    beta, theta = lanczos.lmax(lambda v: gsp @ (asp @ (gtsp @ v)), v0)
    A = _upload(chf, p)
    G = chf.fsai_setup(A, chf.pattern_lower(A))
    gbeta, gtheta = chf.lmax_lanczos(A, G, dev(v0))
    assert abs(gtheta - theta) < 1e-9 * theta
    b_ = rhs(3, p.ndof)
    x0 = np.random.default_rng(4).standard_normal(p.ndof)
    want = chebyshev.cheb4(lambda v: asp @ v, lambda v: gtsp @ (gsp @ v), b_, None if x_is_zero else x0, beta,
                           degree, x_is_zero=x_is_zero)
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda") if x_is_zero else dev(x0)
    work = torch.zeros(3 * p.ndof, dtype=torch.float64, device="cuda")
    chf.cheb4_smooth(A, G, beta, degree, dev(b_), x, x_is_zero=x_is_zero, work=work)
    assert rel_err(host(x), want) < 1e-12
    # the allocation-free entry point runs the same kernels
    x2 = torch.zeros(p.ndof, dtype=torch.float64, device="cuda") if x_is_zero else dev(x0)
    chf.cheb4_smooth_noalloc(A, G, beta, degree, dev(b_), x2, x_is_zero=x_is_zero)
    torch.cuda.synchronize()
    assert torch.equal(x, x2)


def test_vbsr_uniform_only_calls_refuse(chf):
    p = make_vb_problem(6, 2, 2, 2, 3, seed=0)
    A = _upload(chf, p)
    for call in (lambda: chf.pattern_adaptive(A, 4), lambda: chf.levels_create(A),
                 lambda: chf.fsai_setup(A, chf.pattern_lower(A), g_store=chf.F32)):
        with pytest.raises(chf.ChfError) as ei:
            call()
        assert ei.value.code == -1


def test_vbsr_not_spd_reports_row(chf):
    p = make_vb_problem(6, 2, 2, 2, 3, seed=0)
    vals = p.vals.copy()
    k = 14                                     # zero the diagonal block of row 14
    e = int(p.rowptr[k] + np.searchsorted(p.colidx[p.rowptr[k]:p.rowptr[k + 1]], k))
    vals[p.voff[e]:p.voff[e + 1]] = 0.0
    A = chf.vbsr_create(p.nb, p.bsize, p.rowptr, p.colidx, vals)
    P = chf.pattern_from_csr(p.nb, np.arange(p.nb + 1, dtype=np.int64), np.arange(p.nb, dtype=np.int32))
    with pytest.raises(chf.ChfError) as ei:
        chf.fsai_setup(A, P)
    assert ei.value.code == -3 and ei.value.bad_row == k
