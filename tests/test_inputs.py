"""Pins for the seeded input generator (block counts, closed-form stencils,
structure of R and of the prolongator)."""
import numpy as np
import pytest
import scipy.sparse as sp

from problems import make_problem, prolongator, prolongator_1d, stencil_matrix


def _row_stencil(d, n, ix, iy):
    i = ix + n * iy
    row = d.getrow(i)
    out = {}
    for j, v in zip(row.indices, row.data):
        out[(j % n - ix, j // n - iy)] = v
    return out


def test_biharmonic_interior_stencil():
    # (4 - s)^2 = 16 - 8 s + s^2 with s the sum of the four grid shifts:
    # centre 16 + 4 = 20, axis -8, diagonal 2, distance-2 axis 1 (13 points).
    st = _row_stencil(stencil_matrix(9, 2, 2), 9, 4, 4)
    want = {(0, 0): 20, (1, 0): -8, (-1, 0): -8, (0, 1): -8, (0, -1): -8,
            (1, 1): 2, (1, -1): 2, (-1, 1): 2, (-1, -1): 2,
            (2, 0): 1, (-2, 0): 1, (0, 2): 1, (0, -2): 1}
    assert st == want


def test_triharmonic_interior_stencil():
    # (4 - s)^3 = 64 - 48 s + 12 s^2 - s^3; counting lattice walks gives centre
    # 112, axis -57, 12, -1 at distances 1, 2, 3, diagonal 24 and knight -3.
    st = _row_stencil(stencil_matrix(11, 2, 3), 11, 5, 5)
    assert len(st) == 25
    assert st[(0, 0)] == 112
    for v in [(1, 0), (-1, 0), (0, 1), (0, -1)]:
        assert st[v] == -57
    for v in [(2, 0), (0, -2)]:
        assert st[v] == 12
    for v in [(3, 0), (0, 3)]:
        assert st[v] == -1
    for v in [(1, 1), (-1, 1)]:
        assert st[v] == 24
    for v in [(2, 1), (1, -2), (-2, -1)]:
        assert st[v] == -3


def test_3d_biharmonic_stencil_points():
    st = stencil_matrix(7, 3, 2)
    i = 3 + 7 * 3 + 49 * 3
    row = st.getrow(i)
    assert row.nnz == 25
    assert dict(zip(row.indices, row.data))[i] == 36 + 6


@pytest.mark.parametrize("n,dim,power,nnzb", [
    (32, 2, 2, 12676), (512, 2, 2, 3397636), (256, 2, 3, 1624084), (64, 3, 2, 6382336)])
def test_block_counts(n, dim, power, nnzb):
    assert stencil_matrix(n, dim, power).nnz == nnzb


@pytest.mark.parametrize("n,nlower", [(32, 6850), (512, 1829890)])
def test_lower_counts(n, nlower):
    assert sp.tril(stencil_matrix(n, 2, 2)).nnz == nlower


def test_blocks_structure():
    p = make_problem(5, 2, 4, 2, seed=3)
    a = p.to_scipy().toarray()
    assert np.array_equal(a, a.T)
    # R_i = Q_i diag(exp u_i): Q orthogonal, singular values in [e^-1, e]
    for i in range(p.nb):
        s = np.linalg.svd(p.rfac[i], compute_uv=False)
        assert s.max() <= np.e * (1 + 1e-12) and s.min() >= np.exp(-1) * (1 - 1e-12)
    # A_ii = D_ii R_i^T R_i = D_ii diag(exp(2 u_i)) is diagonal
    for i in range(p.nb):
        blk = p.vals[p.rowptr[i] + np.searchsorted(p.colidx[p.rowptr[i]:p.rowptr[i + 1]], i)]
        assert np.allclose(blk, np.diag(np.diag(blk)), atol=1e-12 * abs(blk).max())
    assert np.all(np.linalg.eigvalsh(a) > 0)


def test_seed_determinism():
    p1 = make_problem(4, 2, 3, 2, seed=11)
    p2 = make_problem(4, 2, 3, 2, seed=11)
    p3 = make_problem(4, 2, 3, 2, seed=12)
    assert np.array_equal(p1.vals, p2.vals)
    assert not np.array_equal(p1.vals, p3.vals)


def test_prolongator_weights():
    p1 = prolongator_1d(4, boundary="zero_ghost").toarray()
    assert p1.shape == (8, 4)
    assert np.allclose(p1.sum(axis=1), [0.75, 1, 1, 1, 1, 1, 1, 0.75])
    assert p1[2, 1] == 0.75 and p1[2, 0] == 0.25 and p1[3, 2] == 0.25
    d1 = prolongator_1d(4).toarray()
    # Dirichlet-consistent linear interpolation differs only next to the
    # boundary: t = -1/4 between the boundary point -3/4 (value 0) and cell 0
    assert abs(d1[0, 0] - 2.0 / 3.0) < 1e-15 and abs(d1[7, 3] - 2.0 / 3.0) < 1e-15
    assert np.array_equal(d1[1:7], p1[1:7])
    p2 = prolongator(4, 2)
    assert p2.shape == (64, 16)
    assert np.allclose(p2.toarray(), np.kron(d1, d1))


def _fine_coords(nc):
    return np.array([i // 2 - 0.25 if i % 2 == 0 else i // 2 + 0.25 for i in range(2 * nc)])


@pytest.mark.parametrize("order", [2, 4])
def test_prolongator_reproduces_polynomials(order):
    # interior rows reproduce every polynomial of degree < order; rows next to
    # a boundary reproduce those that vanish at the boundary point (-3/4 on
    # the left, nc - 1/4 on the right), the Dirichlet condition of the grid
    nc = 12
    p = prolongator_1d(nc, order).toarray()
    xc = np.arange(nc, dtype=float)
    tf = _fine_coords(nc)
    reach = order // 2 + 1          # fine rows within this many coarse cells see a boundary
    inner = [f for f in range(2 * nc) if reach <= tf[f] <= nc - 1 - reach]
    rng = np.random.default_rng(order)
    for deg in range(order):
        c = rng.standard_normal(deg + 1)
        poly = np.polynomial.Polynomial(c)
        assert np.allclose((p @ poly(xc))[inner], poly(tf)[inner], rtol=0, atol=1e-12 * np.abs(poly(tf)).max())
    for deg in range(order - 1):
        r = np.polynomial.Polynomial(rng.standard_normal(deg + 1))
        for root, near in ((-0.75, tf < reach + 1), (nc - 0.25, tf > nc - 2 - reach)):
            q = np.polynomial.Polynomial([-root, 1.0]) * r       # degree deg + 1 <= order - 1
            got, want = p @ q(xc), q(tf)
            assert np.allclose(got[near], want[near], rtol=0, atol=1e-11 * np.abs(want).max())
    # a polynomial that does not vanish at the boundary is not reproduced there
    ones = p @ np.ones(nc)
    assert ones[0] < 1 - 1e-3 and ones[-1] < 1 - 1e-3


def test_cubic_interior_weights():
    p = prolongator_1d(8, 4).toarray() * 128
    assert np.allclose(p[8, 2:6], [-5, 35, 105, -7])      # fine 2I, I = 4: cells I-2 .. I+1
    assert np.allclose(p[9, 3:7], [-7, 105, 35, -5])      # fine 2I+1: cells I-1 .. I+2
