"""GPU parity of the core path against the oracle, through the C ABI:
SpMV/residual, block-FSAI set-up, fourth-kind smoother, Lanczos bound and
error paths. Sizes span several SpMV slices with a ragged tail; block sizes
1, 3, 10 and 21."""
import numpy as np
import pytest

from oracle import chebyshev, fsai, lanczos
from oracle.bsr import from_problem
from problems import lanczos_starts, make_problem, rhs
from tests.helpers import dev, host, rel_err, upload

pytestmark = pytest.mark.gpu

CASES = [(7, 2, 1, 2), (7, 2, 3, 2), (13, 2, 10, 2), (9, 2, 21, 3), (5, 3, 10, 2), (32, 2, 10, 2)]


@pytest.fixture(scope="module")
def chf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2509_06744_amd as m
    m.lib()
    return m


# CHF_SPMV_SPLIT_BELOW: "0" keeps every matrix on the one-wavefront-per-slice
# kernel, "1000000000" sends every matrix to the split kernel (one workgroup
# per slice), so both SpMV kernels are checked at every size
SPLIT = ["0", "1000000000"]


@pytest.mark.parametrize("n,dim,b,pw", CASES)
@pytest.mark.parametrize("split_below", SPLIT)
def test_bsr_roundtrip_and_spmv(chf, n, dim, b, pw, split_below, monkeypatch):
    monkeypatch.setenv("CHF_SPMV_SPLIT_BELOW", split_below)
    p = make_problem(n, dim, b, pw, seed=1)
    A = upload(p)
    rp, ci, vals = chf.bsr_export(A)
    assert np.array_equal(rp, p.rowptr) and np.array_equal(ci, p.colidx) and np.array_equal(vals, p.vals)
    rng = np.random.default_rng(2)
    x = rng.standard_normal(p.ndof)
    bv = rng.standard_normal(p.ndof)
    ref = p.to_scipy() @ x
    y = dev(np.zeros(p.ndof))
    chf.bsr_spmv(A, dev(x), y)
    assert rel_err(host(y), ref) < 1e-14
    chf.bsr_spmv(A, dev(x), y, bvec=dev(bv))
    assert rel_err(host(y), bv - ref) < 1e-13
    # FP32 storage, FP32 vectors
    import torch
    y32 = torch.zeros(p.ndof, dtype=torch.float32, device="cuda")
    chf.bsr_spmv(A, dev(x, torch.float32), y32, dtype=chf.F32)
    assert rel_err(host(y32), ref) < 2e-5


@pytest.mark.parametrize("n,dim,b,pw", CASES)
def test_fsai_lower_pattern(chf, n, dim, b, pw):
    p = make_problem(n, dim, b, pw, seed=0)
    a = from_problem(p)
    A = upload(p)
    P = chf.pattern_lower(A)
    prow, pcol = chf.pattern_export(P)
    oprow, opcol = fsai.pattern_lower(a)
    assert np.array_equal(prow, oprow) and np.array_equal(pcol, opcol)
    G = chf.fsai_setup(A, P)
    g = chf.fsai_export(G, len(pcol), b)
    want = fsai.fsai(a, oprow, opcol).vals
    assert rel_err(g, want) < 1e-12


def test_fsai_full_pattern_and_diagonal(chf):
    p = make_problem(4, 2, 3, 2, seed=3)
    a = from_problem(p)
    A = upload(p)
    nb = p.nb
    prow = np.concatenate([[0], np.cumsum(np.arange(1, nb + 1))])
    pcol = np.concatenate([np.arange(k + 1) for k in range(nb)])
    G = chf.fsai_setup(A, chf.pattern_from_csr(nb, prow, pcol))
    g = chf.fsai_export(G, len(pcol), 3)
    gd = type(a)(prow, pcol, g, 3).dense()
    ainv = np.linalg.inv(a.dense())
    assert rel_err(gd.T @ gd, ainv) < 1e-12
    dprow, dpcol = fsai.pattern_diagonal(nb)
    G = chf.fsai_setup(A, chf.pattern_from_csr(nb, dprow, dpcol))
    g = chf.fsai_export(G, nb, 3)
    for k in range(nb):
        assert rel_err(g[k].T @ g[k], np.linalg.inv(a.block(k, k))) < 1e-12


@pytest.mark.parametrize("n,dim,b,pw", CASES[1:])
@pytest.mark.parametrize("degree", [1, 3, 4])
@pytest.mark.parametrize("x_is_zero", [False, True])
@pytest.mark.parametrize("split_below", SPLIT)
def test_cheb4_smoother(chf, n, dim, b, pw, degree, x_is_zero, split_below, monkeypatch):
    import torch
    monkeypatch.setenv("CHF_SPMV_SPLIT_BELOW", split_below)
    p = make_problem(n, dim, b, pw, seed=0)
    a = from_problem(p)
    og = fsai.fsai(a, *fsai.pattern_lower(a))
    asp, gsp = a.scipy(), og.scipy()
    gtsp = gsp.T.tocsr()
    beta, _ = lanczos.lmax(lambda v: gsp @ (asp @ (gtsp @ v)), lanczos_starts(0, [p.ndof])[0])
    rng = np.random.default_rng(degree)
    b_ = rhs(0, p.ndof)
    x0 = np.zeros(p.ndof) if x_is_zero else rng.standard_normal(p.ndof)
    want = chebyshev.cheb4(lambda v: asp @ v, lambda v: gtsp @ (gsp @ v), b_, x0, beta, degree,
                           x_is_zero=x_is_zero)
    A = upload(p)
    G = chf.fsai_setup(A, chf.pattern_lower(A))
    x = dev(x0 if not x_is_zero else np.full(p.ndof, np.nan))
    work = torch.empty(3 * p.ndof, dtype=torch.float64, device="cuda")
    chf.cheb4_smooth(A, G, beta, degree, dev(b_), x, x_is_zero=x_is_zero, work=work)
    assert rel_err(host(x), want) < 1e-12


def test_lanczos_bound(chf):
    p = make_problem(16, 2, 10, 2, seed=0)
    a = from_problem(p)
    og = fsai.fsai(a, *fsai.pattern_lower(a))
    asp, gsp = a.scipy(), og.scipy()
    gtsp = gsp.T.tocsr()
    v0 = lanczos_starts(0, [p.ndof])[0]
    want, wtheta = lanczos.lmax(lambda v: gsp @ (asp @ (gtsp @ v)), v0)
    A = upload(p)
    G = chf.fsai_setup(A, chf.pattern_lower(A))
    beta, theta = chf.lmax_lanczos(A, G, dev(v0))
    assert abs(theta - wtheta) < 1e-9 * wtheta
    assert abs(beta - 1.01 * theta) < 1e-15 * beta
    bm = (gsp @ asp @ gtsp).toarray()
    assert beta >= np.linalg.eigvalsh(bm).max()


# Negating A_kk makes the local system of row k indefinite, first at block k's
# first pivot; rows below k do not contain block k, so k is the reported row.
# With '256,1' every row goes through the tiled solver, which factors pairs of
# tile columns: at b = 10 the failing pivot of row 1 (row 10 of a 20-wide
# system) lies in tile column 0, the first of a pair, and that of row 17 (row
# 50 of a 60-wide system) in tile column 3, the second of a pair. With
# '256,1,0' every row goes through the register-resident kernel, which meets
# the failing pivot in the inverse of its last diagonal tile.
@pytest.mark.parametrize("b,k", [(3, 17), (10, 1), (10, 17)])
@pytest.mark.parametrize("config", [None, "256,1", "256,1,0"])
def test_error_not_spd_reports_row(chf, b, k, config, monkeypatch):
    if config:
        monkeypatch.setenv("CHF_FSAI_CONFIG", config)
    p = make_problem(6, 2, b, 2, seed=0)
    vals = p.vals.copy()
    e = p.rowptr[k] + np.searchsorted(p.colidx[p.rowptr[k]:p.rowptr[k + 1]], k)
    vals[e] = -vals[e]
    A = chf.bsr_create(p.nb, p.b, p.rowptr, p.colidx, vals)
    with pytest.raises(chf.ChfError) as ei:
        chf.fsai_setup(A, chf.pattern_lower(A))
    assert ei.value.code == -3 and ei.value.bad_row == k


def test_error_bad_inputs(chf):
    p = make_problem(4, 2, 3, 2, seed=0)
    vals = p.vals.copy()
    vals[3, 1, 1] = np.nan
    with pytest.raises(chf.ChfError) as ei:
        chf.bsr_create(p.nb, p.b, p.rowptr, p.colidx, vals)
    assert ei.value.code == -1
    # unsorted / upper / missing diagonal patterns
    with pytest.raises(chf.ChfError):
        chf.pattern_from_csr(2, [0, 1, 3], [0, 1, 0])
    with pytest.raises(chf.ChfError):
        chf.pattern_from_csr(2, [0, 2, 3], [0, 1, 1])
    with pytest.raises(chf.ChfError):
        chf.pattern_from_csr(2, [0, 1, 2], [0, 0])
    A = upload(p)
    G = chf.fsai_setup(A, chf.pattern_lower(A))
    import torch
    z = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    with pytest.raises(chf.ChfError):
        chf.cheb4_smooth(A, G, -1.0, 3, z, z, work=torch.zeros(3 * p.ndof, dtype=torch.float64, device="cuda"))
    with pytest.raises(chf.ChfError):
        chf.cheb4_smooth(A, G, 1.0, 0, z, z, work=torch.zeros(3 * p.ndof, dtype=torch.float64, device="cuda"))


def test_error_misaligned_vector(chf):
    """At b = 10 the products read x in pairs: a vector that does not start on
    a 16-byte (FP64) boundary is rejected on the host before any launch; the
    same product on an aligned copy runs."""
    import torch
    p = make_problem(4, 2, 10, 2, seed=0)
    A = upload(p)
    buf = torch.zeros(p.ndof + 2, dtype=torch.float64, device="cuda")
    x_bad = buf[1:1 + p.ndof]
    assert x_bad.data_ptr() % 16 == 8
    y = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    with pytest.raises(chf.ChfError) as ei:
        chf.bsr_spmv(A, x_bad, y)
    assert ei.value.code == -1
    chf.bsr_spmv(A, buf[2:2 + p.ndof], y)
    torch.cuda.synchronize()


def test_empty_matrix(chf):
    A = chf.bsr_create(0, 3, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros((0, 3, 3)))
    assert A.info() == (0, 3, 0)
    P = chf.pattern_lower(A)
    G = chf.fsai_setup(A, P)
    assert G is not None


def test_run_twice_bit_identical(chf):
    import torch
    p = make_problem(20, 2, 10, 2, seed=4)
    A = upload(p)
    G = chf.fsai_setup(A, chf.pattern_lower(A))
    b_ = dev(rhs(4, p.ndof))
    outs = []
    for _ in range(2):
        x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
        w = torch.zeros(3 * p.ndof, dtype=torch.float64, device="cuda")
        chf.cheb4_smooth(A, G, 3.0, 4, b_, x, x_is_zero=True, work=w)
        outs.append(host(x))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("n,dim,b,pw,tmax", [(9, 2, 10, 2, 8), (4, 3, 10, 2, 23), (8, 2, 3, 2, 12), (7, 2, 1, 2, 20)])
@pytest.mark.parametrize("config", ["256,1", "256,48", "64,0", "128,0", "256,1,0", "256,48,96"])
def test_fsai_configs_match_oracle(chf, n, dim, b, pw, tmax, config, monkeypatch):
    """Every solver configuration (width, tiled-MFMA threshold, register-
    resident threshold) gives the oracle's G; '256,1' sends every row through
    the tiled MFMA path, '256,1,0' every row of at most 240 through the
    register-resident kernel (from 1 to 15 tiles), and the 3D t_max = 23 case
    has local systems up to 240 wide."""
    from oracle import adaptive
    p = make_problem(n, dim, b, pw, seed=0)
    a = from_problem(p)
    prow, pcol = adaptive.adaptive_pattern(a, tmax)
    monkeypatch.setenv("CHF_FSAI_CONFIG", config)
    A = upload(p)
    G = chf.fsai_setup(A, chf.pattern_from_csr(p.nb, prow, pcol))
    g = chf.fsai_export(G, len(pcol), b)
    want = fsai.fsai(a, prow, pcol).vals
    assert rel_err(g, want) < 1e-12
