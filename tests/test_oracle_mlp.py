"""Pins for the MLP oracle: backprop against central finite differences and
closed-form features on the unrotated problem D (x) I_b."""
import math

import numpy as np

from oracle import mlp
from oracle.bsr import from_problem
from problems import make_problem, mlp_init


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = mlp_init(3).astype(np.float64)
    o1 = mlp.H * mlp.NIN
    o2 = o1 + mlp.H + mlp.H * mlp.H
    p[o1:o1 + 64] = 0.1 * rng.standard_normal(64)     # nonzero biases
    p[o2:o2 + 64] = 0.1 * rng.standard_normal(64)
    x = rng.standard_normal((40, mlp.NIN))
    y = (rng.uniform(size=40) < 0.4).astype(np.float64)
    lval, g = mlp.loss_grad(p, x, y)
    assert abs(lval - mlp.loss(p, x, y)) < 1e-14
    idx = rng.choice(mlp.NPARAM, 200, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd = (mlp.loss(p + e, x, y) - mlp.loss(p - e, x, y)) / (2 * h)
        assert abs(fd - g[i]) < 1e-7 + 1e-5 * abs(g[i]), i


def test_loss_closed_form_zero_net():
    p = np.zeros(mlp.NPARAM)
    x = np.ones((5, mlp.NIN))
    y = np.array([0, 1, 1, 0, 1.0])
    assert abs(mlp.loss(p, x, y) - math.log(2)) < 1e-15


def test_features_closed_form_unrotated():
    # with R = I: A_ij = D_ij I_b, so f0 = |D_kc| / sqrt(D_kk D_cc),
    # f1 = |D_ck / D_cc| sqrt(b), f2..f4 the grid offset of c from k,
    # f5 = -b log(1 - D_kc^2 / (D_kk D_cc))
    n, b = 6, 3
    p = make_problem(n, 2, b, 2, seed=0, rotate=False)
    a = from_problem(p)
    d = p.dstencil.toarray()
    crow, ccol, feats = mlp.features(a, n, n, rows=[14, 21, 35])
    for k, (cand, f) in feats.items():
        for c, fc in zip(cand, f):
            dkc, dkk, dcc = d[k, c], d[k, k], d[c, c]
            assert abs(fc[0] - abs(dkc) / math.sqrt(dkk * dcc)) < 1e-12
            assert abs(fc[1] - abs(dkc / dcc) * math.sqrt(b)) < 1e-12
            assert (fc[2], fc[3], fc[4]) == (c % n - k % n, c // n - k // n, 0)
            want = -b * math.log1p(-dkc * dkc / (dkk * dcc))
            assert abs(fc[5] - want) < 1e-12 * max(1.0, want)


def test_topk_ties_to_smaller_column():
    crow = np.array([0, 0, 1, 3])
    ccol = np.array([0, 1, 0])
    score = np.array([0.5, 2.0, 2.0])
    prow, pcol = mlp.topk_pattern(crow, ccol, score, 1)
    assert list(pcol[prow[2]:prow[3]]) == [0, 2]
    assert list(pcol[prow[1]:prow[2]]) == [0, 1]
    assert list(pcol[prow[0]:prow[1]]) == [0]


def test_a2_candidates_match_scipy_structure():
    # candidates = strictly lower part of the block pattern of A^2, formed here
    # by SciPy's sparse product of the 0/1 block structure (no cancellation)
    import scipy.sparse as sp
    for n, dim, b in [(7, 2, 2), (4, 3, 1)]:
        p = make_problem(n, dim, b, 2, seed=1)
        a = from_problem(p)
        s = sp.csr_matrix((np.ones(p.nnzb), p.colidx, p.rowptr), shape=(p.nb, p.nb))
        s2 = sp.tril(s @ s, k=-1, format="csr")
        s2.sort_indices()
        crow, ccol = mlp.a2_candidates(a)
        assert np.array_equal(crow, s2.indptr.astype(np.int64))
        assert np.array_equal(ccol, s2.indices.astype(np.int64))


def test_labels_hand_built():
    # rows 0..2; row 1 has candidates {0}, row 2 has {0, 1};
    # pattern P_1 = {1}, P_2 = {0, 2}
    crow = np.array([0, 0, 1, 3])
    ccol = np.array([0, 0, 1])
    prow = np.array([0, 1, 2, 4])
    pcol = np.array([0, 1, 0, 2])
    assert list(mlp.labels(crow, ccol, prow, pcol)) == [0.0, 1.0, 0.0]


def test_adam_closed_forms():
    """Adam from zero moments: with bias correction the first move is
    lr g / (|g| + eps) whatever beta1, beta2; a constant gradient keeps
    m_hat = g and v_hat = g^2, so every move is the same; a gradient that
    flips sign at step 2 gives m_hat = -(1 - beta1) / (1 + beta1) g and
    v_hat = g^2."""
    rng = np.random.default_rng(3)
    n = 50
    p0 = rng.standard_normal(n)
    g = rng.standard_normal(n) * 10.0 ** rng.uniform(-6, 1, n)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    z = np.zeros(n)
    p1, m1, v1 = mlp.adam_step(p0, g, z, z, 1, lr, b1, b2, eps)
    step = lr * g / (np.abs(g) + eps)
    assert np.allclose(p1, p0 - step, rtol=0, atol=1e-15)
    p, m, v = p0, z, z
    for t in range(1, 6):
        p, m, v = mlp.adam_step(p, g, m, v, t, lr, b1, b2, eps)
    assert np.allclose(p, p0 - 5 * step, rtol=0, atol=1e-14)
    p2, _, _ = mlp.adam_step(p1, -g, m1, v1, 2, lr, b1, b2, eps)
    want = p1 + lr * ((1 - b1) / (1 + b1)) * g / (np.abs(g) + eps)
    assert np.allclose(p2, want, rtol=0, atol=1e-14)
    # a zero gradient leaves the parameter where it is
    pz, _, _ = mlp.adam_step(p0, z, z, z, 1, lr, b1, b2, eps)
    assert np.array_equal(pz, p0)
