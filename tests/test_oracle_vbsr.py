"""Pins for the variable-block oracle (Def. 2.1 with unequal m_i): the
printed size of Ex. 5.1, SPD structure of the generator, Lemma 2.1's
diag(G A G^T) = I with mixed block sizes, the exact inverse factor for a full
lower pattern, block Jacobi for the diagonal pattern, agreement with the
uniform-block oracle when all m_i are equal, and the smoother's spectral
definition on a variable-block operator."""
import numpy as np
import pytest

from oracle import chebyshev, fsai
from oracle import vbsr
from oracle.bsr import Bsr
from problems import make_vb_problem, vb_block_sizes


def test_ex51_dof_count():
    # 128 x 128 patches, p = 2 (6 functions) inside and p = 3 (10) on the
    # boundary patches: 15,876 x 6 + 508 x 10 = 100,336 unknowns
    m = vb_block_sizes(128, 2, 2, 3)
    assert int(m.sum()) == 100336 and int((m == 10).sum()) == 508 and int((m == 6).sum()) == 15876
    assert int(vb_block_sizes(5, 3, 1, 2).sum()) == 27 * 4 + 98 * 10


def test_generator_spd_and_diagonal_blocks():
    p = make_vb_problem(6, 2, 2, seed=2)
    a = vbsr.from_problem(p)
    d = a.dense()
    assert np.abs(d - d.T).max() < 1e-12 * np.abs(d).max()
    assert np.linalg.eigvalsh(d).min() > 0
    for i in (0, 7, 14):
        blk = a.block(i, i)
        assert np.abs(blk - np.diag(np.diag(blk))).max() < 1e-12 * np.abs(blk).max()


@pytest.fixture(scope="module")
def vb_small():
    p = make_vb_problem(7, 2, 2, seed=1)
    return p, vbsr.from_problem(p)


def _gdense(g):
    return g.dense()


def test_diag_gagt_identity_mixed_sizes(vb_small):
    # Lemma 2.1: diag_B(G A G^T) = I, each diagonal block of its own size m_k
    p, a = vb_small
    prow, pcol = fsai.pattern_lower(a)
    g = vbsr.fsai(a, prow, pcol)
    m = _gdense(g) @ a.dense() @ _gdense(g).T
    boff = a.boff
    for k in range(a.nb):
        blk = m[boff[k]:boff[k + 1], boff[k]:boff[k + 1]]
        assert np.abs(blk - np.eye(blk.shape[0])).max() < 1e-12


def test_full_lower_pattern_gives_inverse_cholesky(vb_small):
    p, a = vb_small
    prow = np.concatenate([[0], np.cumsum(np.arange(1, a.nb + 1))]).astype(np.int64)
    pcol = np.concatenate([np.arange(k + 1) for k in range(a.nb)]).astype(np.int64)
    gd = _gdense(vbsr.fsai(a, prow, pcol))
    ad = a.dense()
    assert np.abs(gd.T @ gd - np.linalg.inv(ad)).max() < 1e-12 * np.abs(np.linalg.inv(ad)).max()
    assert np.abs(gd - np.linalg.inv(np.linalg.cholesky(ad))).max() < 1e-12 * np.abs(gd).max()


def test_diagonal_pattern_is_block_jacobi(vb_small):
    p, a = vb_small
    prow, pcol = fsai.pattern_diagonal(a.nb)
    g = vbsr.fsai(a, prow, pcol)
    for k in range(a.nb):
        gk = g.block(k, k)
        assert np.abs(gk.T @ gk - np.linalg.inv(a.block(k, k))).max() < 1e-12 * np.abs(gk).max() ** 2


def test_equal_blocks_match_uniform_oracle():
    # p_interior = p_boundary: every m_i = 6, so the variable-block code must
    # reproduce the uniform-block oracle on the same matrix
    p = make_vb_problem(6, 2, 2, p_interior=2, p_boundary=2, seed=3)
    a = vbsr.from_problem(p)
    b = 6
    ub = Bsr(p.rowptr, p.colidx.astype(np.int64), p.vals.reshape(-1, b, b), b)
    prow, pcol = fsai.pattern_lower(ub)
    gu = fsai.fsai(ub, prow, pcol)
    gv = vbsr.fsai(a, prow, pcol)
    assert np.abs(gv.vals - gu.vals.ravel()).max() < 1e-13 * np.abs(gu.vals).max()


@pytest.mark.parametrize("k", [1, 3, 4])
def test_smoother_spectral_definition_variable_blocks(vb_small, k):
    p, a = vb_small
    prow, pcol = fsai.pattern_lower(a)
    gd = _gdense(vbsr.fsai(a, prow, pcol))
    ad = a.dense()
    lmax = np.linalg.eigvalsh(gd @ ad @ gd.T).max()
    rng = np.random.default_rng(k)
    b, x0 = rng.standard_normal((2, a.ndof))
    asp = a.scipy()
    x = chebyshev.cheb4(lambda v: asp @ v, lambda v: gd.T @ (gd @ v), b, x0, 1.01 * lmax, k)
    xs = chebyshev.cheb4_spectral(gd, ad, b, x0, 1.01 * lmax, k)
    assert np.abs(x - xs).max() < 1e-10 * np.abs(xs).max()
