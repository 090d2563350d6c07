"""Pins for the oracle's Algorithm 1 (adaptive block-FSAI): Lemma 2.4 against
a brute-force rebuild, greedy optimality against brute-force Kaporin numbers,
monotone Kaporin decrease, and the invariance of patterns under the block
rotation R (the scalar problem D gives the same pattern)."""
import math

import numpy as np
import pytest

from oracle import adaptive, fsai
from oracle.bsr import Bsr, from_problem
from problems import make_problem


@pytest.fixture(scope="module")
def prob():
    return from_problem(make_problem(5, 2, 3, 2, seed=2))


def _g_dense(a, rows_patterns):
    prow = [0]
    pcol = []
    for pk in rows_patterns:
        pcol.extend(pk)
        prow.append(len(pcol))
    return fsai.fsai(a, np.array(prow), np.array(pcol)).dense()


def test_lemma_2_4_against_rebuild(prob):
    a = prob
    rng = np.random.default_rng(0)
    for k in [7, 12, 18, 24]:
        pk = [k]
        for _ in range(3):
            cand = adaptive.candidates(a, k, pk)
            g = adaptive.gains(a, k, pk, cand)
            _, s_kk, _ = fsai.fsai_row(a, k, pk)
            base = np.linalg.slogdet(s_kk)[1]
            for c, gc in zip(cand, g):
                _, s_new, _ = fsai.fsai_row(a, k, sorted(pk + [c]))
                # rho_c = det((F^(c) A F^(c)T)_kk) / det((F A F^T)_kk)
                assert abs(-(np.linalg.slogdet(s_new)[1] - base) - gc) < 1e-9 * max(1.0, abs(gc))
            pk = sorted(pk + [cand[int(rng.integers(len(cand)))]])


def test_gain_forms_agree(prob):
    a = prob
    for k in [9, 20]:
        pk = [k, k - 1]
        cand = adaptive.candidates(a, k, pk)
        assert np.allclose(adaptive.gains(a, k, pk, cand), adaptive.gains_logdet(a, k, pk, cand),
                           rtol=1e-9, atol=1e-11)


def test_logdet_one_minus_small_and_exact():
    c = np.diag([0.5, 0.25])
    assert abs(adaptive.logdet_one_minus(c) - (math.log(0.5) + math.log(0.75))) < 1e-15
    tiny = np.diag([1e-20, 3e-20])
    assert abs(adaptive.logdet_one_minus(tiny) + 4e-20) < 1e-30
    rng = np.random.default_rng(1)
    x = 0.3 * rng.standard_normal((4, 4))
    cc = x @ x.T / (1.1 * np.linalg.norm(x @ x.T, 2))
    assert abs(adaptive.logdet_one_minus(cc) - np.linalg.slogdet(np.eye(4) - cc)[1]) < 1e-13


def test_candidates_rule(prob):
    a = prob
    k = 18
    pk = [11, 13, 18]
    cand = adaptive.candidates(a, k, pk)
    assert all(c < k and c not in pk for c in cand)
    # every c with a structurally nonzero (F A)_kc is present
    struct = set()
    for j in pk:
        struct |= set(int(c) for c in a.cols(j))
    assert set(cand) == {c for c in struct if c < k and c not in pk}


def test_greedy_choice_minimises_kaporin(prob):
    # Lemma 2.3: beta(GAG^T)^N = prod det S_kk / det A, so enlarging row k by
    # c* must give the smallest Kaporin number among all single enlargements.
    a = prob
    ad = a.dense()
    base = [[j] for j in range(a.nb)]
    for k in [6, 13, 19]:
        pk = [k]
        cand = adaptive.candidates(a, k, pk)
        g = adaptive.gains(a, k, pk, cand)
        cstar, _, _ = adaptive.pick(cand, g)
        kap = {}
        for c in cand:
            pats = [list(p) for p in base]
            pats[k] = sorted([k, c])
            gd = _g_dense(a, pats)
            kap[c] = fsai.kaporin(gd @ ad @ gd.T)
        best = min(kap.values())
        assert kap[cstar] <= best * (1 + 1e-12)


def test_kaporin_decreases_with_steps():
    a = from_problem(make_problem(4, 2, 2, 2, seed=4))
    ad = a.dense()
    prev = math.inf
    for t in range(0, 5):
        prow, pcol = adaptive.adaptive_pattern(a, t)
        g = fsai.fsai(a, prow, pcol).dense()
        kap = fsai.kaporin(g @ ad @ g.T)
        assert kap <= prev * (1 + 1e-12)
        prev = kap


def test_pattern_is_lower_with_diagonal_and_bounded():
    a = from_problem(make_problem(6, 2, 3, 2, seed=0))
    prow, pcol = adaptive.adaptive_pattern(a, 4)
    fsai.check_pattern(a.nb, prow, pcol)
    assert np.max(np.diff(prow)) <= 5


def test_rotation_invariance_of_pattern():
    # A = R^T (D (x) I) R with R block diagonal: every quantity of Lemma 2.4
    # transforms by congruence, rho_c(A) = rho_c(D)^b, so the adaptive pattern
    # of A equals that of the scalar D (with the tie rule).
    n, tmax = 12, 6
    blk = from_problem(make_problem(n, 2, 3, 2, seed=0))
    sca = from_problem(make_problem(n, 2, 1, 2, seed=0, rotate=False))
    p1 = adaptive.adaptive_pattern(blk, tmax)
    p2 = adaptive.adaptive_pattern(sca, tmax)
    assert np.array_equal(p1[0], p2[0]) and np.array_equal(p1[1], p2[1])
    # gains scale by b
    k = 5 + n * 6
    pk = [k, k - 1]
    c1 = adaptive.candidates(blk, k, pk)
    assert c1 == adaptive.candidates(sca, k, pk)
    assert np.allclose(adaptive.gains(blk, k, pk, c1), 3 * adaptive.gains(sca, k, pk, c1), rtol=1e-9)


def test_interior_template():
    # Interior rows of the translation-invariant grid share one offset set.
    n = 14
    sca = from_problem(make_problem(n, 2, 1, 2, seed=0, rotate=False))
    prow, pcol = adaptive.adaptive_pattern(sca, 6)
    offs = set()
    for iy in range(5, n - 2):
        for ix in range(5, n - 5):
            k = ix + n * iy
            row = pcol[prow[k]:prow[k + 1]]
            offs.add(tuple(sorted((int(j) % n - ix, int(j) // n - iy) for j in row)))
    assert len(offs) == 1
