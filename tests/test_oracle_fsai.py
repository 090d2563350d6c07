"""Pins for the oracle's block-FSAI factor (Sec. 2: Def. 2.2, Lemma 2.1,
Remark after Lemma 2.1, Lemma 2.3, Thm. 2.1) and its failure modes."""
import numpy as np
import pytest

from oracle import fsai
from oracle.bsr import from_problem
from problems import make_problem


def _blk(m, i, j, b):
    return m[i * b:(i + 1) * b, j * b:(j + 1) * b]


def _full_lower(nb):
    prow = np.concatenate([[0], np.cumsum(np.arange(1, nb + 1))]).astype(np.int64)
    pcol = np.concatenate([np.arange(k + 1) for k in range(nb)]).astype(np.int64)
    return prow, pcol


@pytest.fixture(scope="module")
def prob():
    return make_problem(4, 2, 3, 2, seed=0)


def test_block_diagonal_identity(prob):
    # Lemma 2.1: diag_B(G A G^T) = I
    a = from_problem(prob)
    g = fsai.fsai(a, *fsai.pattern_lower(a)).dense()
    bm = g @ a.dense() @ g.T
    for i in range(a.nb):
        assert np.abs(_blk(bm, i, i, 3) - np.eye(3)).max() < 1e-13


def test_lemma_2_1_fa_and_faft(prob):
    a = from_problem(prob)
    prow, pcol = fsai.pattern_lower(a)
    f, s = fsai.fsai_f_s(a, prow, pcol)
    fd, ad = f.dense(), a.dense()
    fa, fat = fd @ ad, fd @ ad @ fd.T
    for i in range(a.nb):
        assert np.allclose(_blk(fa, i, i, 3), s[i], rtol=0, atol=1e-11 * abs(s[i]).max())
        assert np.allclose(_blk(fat, i, i, 3), s[i], rtol=0, atol=1e-11 * abs(s[i]).max())
    # Eq. fsai_helper: (FA)[k, P~_k] = 0
    for k in range(a.nb):
        for j in pcol[prow[k]:prow[k + 1] - 1]:
            assert abs(_blk(fa, k, j, 3)).max() < 1e-11 * abs(ad).max()


def test_full_pattern_gives_inverse_cholesky(prob):
    # With the full lower pattern, G is the inverse Cholesky factor of A and
    # G^T G = A^{-1} (the construction G ~ L^{-1} of Sec. 2).
    a = from_problem(prob)
    g = fsai.fsai(a, *_full_lower(a.nb)).dense()
    ad = a.dense()
    ainv = np.linalg.inv(ad)
    assert abs(g.T @ g - ainv).max() < 1e-12 * abs(ainv).max()
    lchol = np.linalg.cholesky(ad)
    assert abs(g - np.linalg.inv(lchol)).max() < 1e-12 * abs(g).max()


def test_diagonal_pattern_is_block_jacobi(prob):
    a = from_problem(prob)
    g = fsai.fsai(a, *fsai.pattern_diagonal(a.nb))
    for k in range(a.nb):
        gk = g.vals[k]
        akk = a.block(k, k)
        assert np.allclose(gk.T @ gk, np.linalg.inv(akk), rtol=1e-13, atol=0)
        assert np.allclose(np.tril(gk), gk)


def test_kaporin_lemma_2_3(prob):
    # beta(G A G^T) = (prod det S_kk / det A)^{1/N}
    a = from_problem(prob)
    prow, pcol = fsai.pattern_lower(a)
    g = fsai.fsai(a, prow, pcol).dense()
    _, s = fsai.fsai_f_s(a, prow, pcol)
    ad = a.dense()
    n = ad.shape[0]
    direct = fsai.kaporin(g @ ad @ g.T)
    lemma = np.exp((sum(np.linalg.slogdet(sk)[1] for sk in s) - np.linalg.slogdet(ad)[1]) / n)
    assert abs(direct - lemma) < 1e-12 * direct
    # Eigenvalue form of Def. 2.3: arithmetic over geometric mean
    ev = np.linalg.eigvalsh(g @ ad @ g.T)
    assert abs(direct - ev.mean() / np.exp(np.log(ev).mean())) < 1e-12 * direct


def test_fsai_optimality_theorem_2_1(prob):
    # Any in-pattern perturbation of G raises the Kaporin number.
    a = from_problem(prob)
    prow, pcol = fsai.pattern_lower(a)
    g = fsai.fsai(a, prow, pcol)
    ad = a.dense()
    k0 = fsai.kaporin(g.dense() @ ad @ g.dense().T)
    rng = np.random.default_rng(5)
    for _ in range(20):
        pert = g.vals + 1e-3 * rng.standard_normal(g.vals.shape) * abs(g.vals).max()
        gp = type(g)(g.rowptr, g.colidx, pert, g.b).dense()
        assert fsai.kaporin(gp @ ad @ gp.T) > k0


def test_pattern_validation():
    prow = np.array([0, 1, 3], dtype=np.int64)
    with pytest.raises(ValueError):
        fsai.check_pattern(2, prow, np.array([0, 1, 0]))     # unsorted
    with pytest.raises(ValueError):
        fsai.check_pattern(2, prow, np.array([0, 0, 1])[[0, 1, 1]])  # diagonal dup
    with pytest.raises(ValueError):
        fsai.check_pattern(2, np.array([0, 1, 2]), np.array([0, 0]))  # row 1 lacks diagonal
    fsai.check_pattern(2, prow, np.array([0, 0, 1]))


def test_not_spd_raises():
    p = make_problem(3, 2, 2, 2, seed=1)
    a = from_problem(p)
    a.vals = a.vals.copy()
    k = 4
    pos = a.rowptr[k] + np.searchsorted(a.cols(k), k)
    a.vals[pos] = -a.vals[pos]
    with pytest.raises(np.linalg.LinAlgError):
        fsai.fsai(a, *fsai.pattern_diagonal(a.nb))
