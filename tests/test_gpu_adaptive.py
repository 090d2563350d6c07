"""GPU Algorithm 1 against the oracle: patterns must match bit for bit (tie
rule included), on small grids for several block sizes, in 3D, and on sampled
rows of the 512 x 512 biharmonic-like workload with t_max = 8."""
import numpy as np
import pytest

from oracle import adaptive, fsai
from oracle.bsr import from_problem
from problems import make_problem, rhs
from tests.helpers import dev, gpu_levels, host, rel_err, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def chf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2509_06744_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("n,dim,b,pw,tmax", [
    (9, 2, 1, 2, 4), (12, 2, 3, 2, 6), (11, 2, 10, 2, 8), (7, 2, 21, 3, 8), (5, 3, 10, 2, 6), (10, 2, 10, 2, 0),
    (6, 2, 2, 2, 20), (6, 3, 10, 2, 23), (8, 2, 16, 2, 5), (5, 2, 32, 2, 3), (7, 2, 10, 2, 1)])
def test_adaptive_pattern_bit_exact(chf, n, dim, b, pw, tmax):
    p = make_problem(n, dim, b, pw, seed=0)
    a = from_problem(p)
    orow, ocol = adaptive.adaptive_pattern(a, tmax)
    A = upload(p)
    P = chf.pattern_adaptive(A, tmax)
    prow, pcol = chf.pattern_export(P)
    assert np.array_equal(prow, orow)
    assert np.array_equal(pcol, ocol)


@pytest.mark.parametrize("n,dim,b,pw,tmax", [(11, 2, 10, 2, 4), (9, 2, 3, 2, 6), (5, 3, 10, 2, 3), (7, 2, 21, 3, 4),
                                               (8, 2, 10, 2, 0)])
def test_adaptive_pattern_from_lower_p0(chf, n, dim, b, pw, tmax):
    """Algorithm 1 started from P0 = lower(A) instead of the diagonal."""
    from oracle import fsai
    p = make_problem(n, dim, b, pw, seed=0)
    a = from_problem(p)
    p0 = fsai.pattern_lower(a)
    orow, ocol = adaptive.adaptive_pattern(a, tmax, p0_pattern=p0)
    A = upload(p)
    P = chf.pattern_adaptive(A, tmax, p0=chf.pattern_lower(A))
    prow, pcol = chf.pattern_export(P)
    assert np.array_equal(prow, orow)
    assert np.array_equal(pcol, ocol)


def test_adaptive_pattern_p0_with_decoupled_blocks(chf):
    """P0 rows holding blocks far from row k (no coupling with k or with the
    rest of P0): they enter as decoupled candidates."""
    p = make_problem(10, 2, 3, 2, seed=1)
    a = from_problem(p)
    rng = np.random.default_rng(4)
    rowptr, cols = [0], []
    for k in range(p.nb):
        extra = sorted(set(int(c) for c in rng.integers(0, k, 2))) if k > 30 else []
        cols.extend(extra + [k])
        rowptr.append(len(cols))
    p0 = (np.array(rowptr, dtype=np.int64), np.array(cols, dtype=np.int64))
    orow, ocol = adaptive.adaptive_pattern(a, 5, p0_pattern=p0)
    A = upload(p)
    P0 = chf.pattern_from_csr(p.nb, p0[0], p0[1].astype(np.int32))
    P = chf.pattern_adaptive(A, 5, p0=P0)
    prow, pcol = chf.pattern_export(P)
    assert np.array_equal(prow, orow)
    assert np.array_equal(pcol, ocol)
    with pytest.raises(chf.ChfError) as ei:      # 3 blocks of P0 + 30 steps > 32
        chf.pattern_adaptive(A, 30, p0=P0)
    assert ei.value.code == -1


def test_adaptive_rotation_invariant_seeds(chf):
    # the pattern of R^T (D (x) I) R does not depend on the seed of R
    pats = []
    for seed in (0, 5):
        p = make_problem(14, 2, 10, 2, seed=seed)
        pats.append(chf.pattern_export(chf.pattern_adaptive(upload(p), 8)))
    assert np.array_equal(pats[0][0], pats[1][0]) and np.array_equal(pats[0][1], pats[1][1])


def test_adaptive_full_size_sampled_rows(chf):
    """512 x 512 patches, b = 10, t_max = 8: sampled rows against the oracle."""
    p = make_problem(512, 2, 10, 2, seed=0)
    a = from_problem(p)
    A = upload(p)
    P = chf.pattern_adaptive(A, 8)
    prow, pcol = chf.pattern_export(P)
    assert prow[-1] <= 9 * p.nb
    rng = np.random.default_rng(0)
    n = 512
    edge = [0, 1, 2, n - 1, n, n + 1, 2 * n + 3, n * n - 1, n * n - n, n * n // 2 + n // 2]
    rows = sorted(set(edge) | set(int(r) for r in rng.integers(0, p.nb, 40)))
    for k in rows:
        want = adaptive.adaptive_row(a, k, 8)
        got = list(pcol[prow[k]:prow[k + 1]])
        assert got == want, f"row {k}"
    # G on the adaptive pattern for sampled rows
    G = chf.fsai_setup(A, P)
    g = chf.fsai_export(G, len(pcol), 10)
    og = fsai.fsai_rows(a, rows, prow, pcol)
    for k in rows:
        assert rel_err(g[prow[k]:prow[k + 1]], og[k]) < 1e-12


def test_adaptive_hierarchy_pcg(chf):
    import torch
    from oracle import multilevel, solver
    from tests.helpers import oracle_levels
    p = make_problem(32, 2, 10, 2, seed=0)
    olv = oracle_levels(p, 3, "adaptive", 4)
    b_ = rhs(0, p.ndof)
    _, oit, _, _ = multilevel.pcg(olv[0].apply_a, lambda r: multilevel.vcycle(olv, 0, r, 3), b_, 1e-8, 100)
    A, L, _, _ = gpu_levels(p, 3, 3, 1, tmax=4)
    for l in range(2):
        _, _, P = chf.levels_get(L, l)
        prow, pcol = chf.pattern_export(P)
        g = olv[l].g
        assert np.array_equal(prow, g.rowptr) and np.array_equal(pcol, g.colidx)
        assert abs(chf.levels_get_beta(L, l) - olv[l].beta) < 1e-9 * olv[l].beta
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    it, hist, tr, _ = chf.pcg_solve(L, dev(b_), x, rtol=1e-8, maxit=100)
    assert abs(it - oit) <= 1 and tr < 1e-7
