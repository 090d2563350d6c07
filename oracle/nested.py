"""Nested block-FSAI with one nesting level (Sec. 2.2).

A_0 = A, F_0 its FSAI factor; A_1 = F_0 A F_0^T and F_1 the FSAI factor of
A_1 (pattern from Algorithm 1 with the same t_max, as in Sec. 5); the
preconditioner is M = F^T S^{-1} F with F = F_1 F_0 and
S = diag_B(F A F^T) (the displayed formula of Sec. 2.2).

The GPU path builds the inner factor for A~_1 = G_0 A G_0^T, where
G_0 = J_0 F_0 is the scaled outer factor, and applies
M = G_0^T G~_1^T G~_1 G_0. Block-FSAI and the ratios rho_c of Algorithm 1 are
invariant under a block-diagonal congruence (A -> D A D^T scales F by
D F D^{-1} and S by D S D^T; rho_c is a ratio of determinants), so this is
the same M and the same inner pattern; `paper_m` and `scaled_m` are the two
forms, compared in the tests.

``triple_product`` is the plain row-by-row definition of G A G^T on the
structural block pattern (no numerical dropping).
"""
from __future__ import annotations

import numpy as np

from . import adaptive, fsai
from .bsr import Bsr


def triple_product(g: Bsr, a: Bsr) -> Bsr:
    """C = G A G^T for block-sparse G and A (same block size), row by row:
    T_i = sum_p G_ip A_p. , then C_ij = sum_q T_iq G_jq^T over the rows j of G
    that have column q. The pattern is structural."""
    b = a.b
    nb = a.nb
    # rows of G holding each column q (the structure of G^T)
    gt_rows = [[] for _ in range(nb)]
    for j in range(nb):
        for e in range(g.rowptr[j], g.rowptr[j + 1]):
            gt_rows[int(g.colidx[e])].append((j, e))
    rowptr = [0]
    cols = []
    vals = []
    for i in range(nb):
        t = {}
        for e in range(g.rowptr[i], g.rowptr[i + 1]):
            p = int(g.colidx[e])
            for f in range(a.rowptr[p], a.rowptr[p + 1]):
                q = int(a.colidx[f])
                t[q] = t.get(q, 0.0) + g.vals[e] @ a.vals[f]
        c = {}
        for q, tq in t.items():
            for j, e in gt_rows[q]:
                c[j] = c.get(j, 0.0) + tq @ g.vals[e].T
        for j in sorted(c):
            cols.append(j)
            vals.append(np.asarray(c[j], dtype=np.float64).reshape(b, b))
        rowptr.append(len(cols))
    return Bsr(np.asarray(rowptr, dtype=np.int64), np.asarray(cols, dtype=np.int64),
               np.asarray(vals, dtype=np.float64).reshape(-1, b, b), b)


def nested(a: Bsr, p0, tmax: int, tau: float = 1.0, p1=None):
    """Outer factor G_0 on pattern p0 = (rowptr, colidx), A~_1 = G_0 A G_0^T,
    inner pattern (Algorithm 1 on A~_1 with t_max, or p1 if given) and inner
    factor G~_1. Returns (g0, a1, p1, g1)."""
    g0 = fsai.fsai(a, *p0)
    a1 = triple_product(g0, a)
    if p1 is None:
        p1 = adaptive.adaptive_pattern(a1, tmax, tau)
    g1 = fsai.fsai(a1, *p1)
    return g0, a1, p1, g1


def apply_m(g0: Bsr, g1: Bsr):
    """v -> G_0^T G~_1^T G~_1 G_0 v with sparse products."""
    s0, s1 = g0.scipy(), g1.scipy()
    s0t, s1t = s0.T.tocsr(), s1.T.tocsr()
    return lambda v: s0t @ (s1t @ (s1 @ (s0 @ v)))


def scaled_m(g0: Bsr, g1: Bsr) -> np.ndarray:
    """Dense M = G_0^T G~_1^T G~_1 G_0 (small problems)."""
    gh = g1.dense() @ g0.dense()
    return gh.T @ gh


def paper_m(a: Bsr, p0, p1) -> np.ndarray:
    """Dense M = F^T S^{-1} F, F = F_1 F_0, S = diag_B(F A F^T), with F_0 on p0
    for A and F_1 on p1 for A_1 = F_0 A F_0^T (unscaled, unit diagonal
    blocks), as displayed in Sec. 2.2. Small problems only."""
    from .bsr import from_scipy
    f0, _ = fsai.fsai_f_s(a, *p0)
    a1 = from_scipy(f0.scipy() @ a.scipy() @ f0.scipy().T, a.b)
    f1, _ = fsai.fsai_f_s(a1, *p1)
    fh = f1.dense() @ f0.dense()
    s = fh @ a.dense() @ fh.T
    b = a.b
    sinv = np.zeros_like(s)
    for k in range(a.nb):
        blk = slice(k * b, (k + 1) * b)
        sinv[blk, blk] = np.linalg.inv(s[blk, blk])
    return fh.T @ sinv @ fh
