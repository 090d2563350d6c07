"""Pins for the oracle's nested block-FSAI (Sec. 2.2, one nesting level):
the triple product against a dense product, the scaled form against the
displayed M = F^T S^{-1} F, invariance of Algorithm 1's pattern under the
block-diagonal congruence, and the two limits of the inner pattern (complete
lower triangle: M = A^{-1}; diagonal: M is the non-nested factor's)."""
import numpy as np
import pytest

from oracle import adaptive, fsai, nested
from oracle.bsr import from_problem
from problems import make_problem


@pytest.fixture(scope="module", params=[(6, 2, 3, 3), (4, 3, 2, 2), (5, 2, 10, 2)])
def case(request):
    n, dim, b, tmax = request.param
    p = make_problem(n, dim, b, 2, seed=0)
    a = from_problem(p)
    p0 = adaptive.adaptive_pattern(a, tmax)
    return a, p0, tmax


def test_triple_product_matches_dense(case):
    a, p0, _ = case
    g0 = fsai.fsai(a, *p0)
    c = nested.triple_product(g0, a)
    want = g0.dense() @ a.dense() @ g0.dense().T
    assert np.abs(c.dense() - want).max() < 1e-12 * np.abs(want).max()
    # every numerically nonzero block lies in the structural pattern
    b = a.b
    blocks = np.abs(want).reshape(a.nb, b, a.nb, b).max(axis=(1, 3)) > 0
    got = np.zeros_like(blocks)
    for i in range(a.nb):
        got[i, c.colidx[c.rowptr[i]:c.rowptr[i + 1]]] = True
    assert not np.any(blocks & ~got)


def test_scaled_form_is_the_displayed_preconditioner(case):
    a, p0, tmax = case
    g0, a1, p1, g1 = nested.nested(a, p0, tmax)
    ms = nested.scaled_m(g0, g1)
    mp = nested.paper_m(a, p0, p1)
    assert np.abs(ms - mp).max() < 1e-10 * np.abs(mp).max()


def test_inner_pattern_invariant_under_scaling(case):
    a, p0, tmax = case
    from oracle.bsr import from_scipy
    f0, _ = fsai.fsai_f_s(a, *p0)
    a1_unscaled = from_scipy(f0.scipy() @ a.scipy() @ f0.scipy().T, a.b)
    g0, a1, p1, g1 = nested.nested(a, p0, tmax)
    q1 = adaptive.adaptive_pattern(a1_unscaled, tmax)
    assert np.array_equal(np.asarray(p1[0]), np.asarray(q1[0]))
    assert np.array_equal(np.asarray(p1[1]), np.asarray(q1[1]))


def test_inner_factor_normalises_diagonal_blocks(case):
    a, p0, tmax = case
    g0, a1, p1, g1 = nested.nested(a, p0, tmax)
    m = g1.dense() @ a1.dense() @ g1.dense().T
    b = a.b
    for k in range(a.nb):
        blk = m[k * b:(k + 1) * b, k * b:(k + 1) * b]
        assert np.abs(blk - np.eye(b)).max() < 1e-10


def test_complete_inner_pattern_gives_exact_inverse():
    p = make_problem(4, 2, 3, 2, seed=1)
    a = from_problem(p)
    p0 = adaptive.adaptive_pattern(a, 2)
    nb = a.nb
    full = (np.concatenate([[0], np.cumsum(np.arange(1, nb + 1))]), np.concatenate([np.arange(k + 1) for k in range(nb)]))
    g0, a1, p1, g1 = nested.nested(a, p0, 0, p1=full)
    m = nested.scaled_m(g0, g1)
    ainv = np.linalg.inv(a.dense())
    assert np.abs(m - ainv).max() < 1e-9 * np.abs(ainv).max()


def test_diagonal_inner_pattern_reduces_to_plain_fsai():
    p = make_problem(5, 2, 3, 2, seed=2)
    a = from_problem(p)
    p0 = adaptive.adaptive_pattern(a, 3)
    g0, a1, p1, g1 = nested.nested(a, p0, 0, p1=fsai.pattern_diagonal(a.nb))
    assert np.abs(g1.vals - np.eye(3)[None]).max() < 1e-12
    m = nested.scaled_m(g0, g1)
    assert np.abs(m - g0.dense().T @ g0.dense()).max() < 1e-12 * np.abs(m).max()
