"""Block-FSAI factor, static patterns and the Kaporin number (paper Sec. 2).

Patterns are CSR arrays (prow int64, pcol int64) over block indices, each row
ascending; a valid pattern is lower triangular and contains the diagonal
(Eq. lower_triangular_pattern), so the diagonal is the last entry of each row.
"""
from __future__ import annotations

import numpy as np

from .bsr import Bsr


def check_pattern(nb: int, prow, pcol) -> None:
    """Raise ValueError unless the pattern is lower triangular with the diagonal
    present and rows strictly ascending (Def. 2.2, Eq. lower_triangular_pattern)."""
    if len(prow) != nb + 1 or prow[0] != 0:
        raise ValueError("bad row pointer")
    for k in range(nb):
        row = pcol[prow[k]:prow[k + 1]]
        if len(row) == 0 or row[-1] != k:
            raise ValueError(f"row {k}: diagonal missing")
        if np.any(np.diff(row) <= 0) or row[0] < 0:
            raise ValueError(f"row {k}: columns not strictly ascending / not lower")


def pattern_lower(a: Bsr):
    """A-priori pattern: the lower block triangle of A, diagonal included (Sec. 2.1)."""
    prow = [0]
    pcol = []
    for k in range(a.nb):
        cols = [int(j) for j in a.cols(k) if j <= k]
        if k not in cols:
            cols.append(k)
        cols = sorted(set(cols))
        pcol.extend(cols)
        prow.append(len(pcol))
    return np.array(prow, dtype=np.int64), np.array(pcol, dtype=np.int64)


def pattern_diagonal(nb: int):
    """The diagonal pattern (block-Jacobi, Remark after Lemma 2.1)."""
    return np.arange(nb + 1, dtype=np.int64), np.arange(nb, dtype=np.int64)


def fsai_row(a: Bsr, k: int, pk):
    """Row k of the block-FSAI matrices of Def. 2.2.

    Returns (F_k on P~_k, S_kk, G blocks on P_k in ascending column order).
    F[k, P~_k] = -A[k, P~_k] A[P~_k, P~_k]^{-1}   (Eq. fsai_f_definition)
    S_kk = A_kk - A[k,P~_k] A[P~_k,P~_k]^{-1} A[P~_k,k]  (Eq. schur_complement_fsai)
    G = J F with J = L_S^{-1}, S_kk = L_S L_S^T, so J^T J = S_kk^{-1}
    (the factor S^{-1/2} after Eq. schur_complement_fsai, read as a Cholesky root).
    """
    b = a.b
    pt = [int(j) for j in pk if j != k]
    akk = a.block(k, k)
    if pt:
        a_kp = a.sub([k], pt)
        a_pp = a.sub(pt, pt)
        a_pp_inv = np.linalg.inv(a_pp)
        f_kp = -a_kp @ a_pp_inv
        s_kk = akk - a_kp @ a_pp_inv @ a_kp.T
    else:
        f_kp = np.zeros((b, 0))
        s_kk = akk.copy()
    s_kk = 0.5 * (s_kk + s_kk.T)
    l_s = np.linalg.cholesky(s_kk)
    jfac = np.linalg.inv(l_s)
    g_kp = jfac @ f_kp
    blocks = [g_kp[:, c * b:(c + 1) * b] for c in range(len(pt))] + [jfac]
    return f_kp, s_kk, np.array(blocks)


def fsai(a: Bsr, prow, pcol) -> Bsr:
    """G = S^{-1/2} F as a block-sparse matrix on the pattern (Def. 2.2)."""
    check_pattern(a.nb, prow, pcol)
    vals = np.zeros((len(pcol), a.b, a.b))
    for k in range(a.nb):
        lo, hi = prow[k], prow[k + 1]
        _, _, g = fsai_row(a, k, pcol[lo:hi])
        vals[lo:hi] = g
    return Bsr(np.asarray(prow, dtype=np.int64), np.asarray(pcol, dtype=np.int64), vals, a.b)


def fsai_rows(a: Bsr, rows, prow, pcol):
    """G blocks for a subset of rows only (for sampled comparisons)."""
    out = {}
    for k in rows:
        lo, hi = prow[k], prow[k + 1]
        out[int(k)] = fsai_row(a, int(k), pcol[lo:hi])[2]
    return out


def fsai_f_s(a: Bsr, prow, pcol):
    """F (block-sparse, unit diagonal) and the block diagonal S (Def. 2.2)."""
    b = a.b
    fvals = np.zeros((len(pcol), b, b))
    svals = np.zeros((a.nb, b, b))
    for k in range(a.nb):
        lo, hi = prow[k], prow[k + 1]
        f_kp, s_kk, _ = fsai_row(a, k, pcol[lo:hi])
        for c in range(hi - lo - 1):
            fvals[lo + c] = f_kp[:, c * b:(c + 1) * b]
        fvals[hi - 1] = np.eye(b)
        svals[k] = s_kk
    f = Bsr(np.asarray(prow, dtype=np.int64), np.asarray(pcol, dtype=np.int64), fvals, b)
    return f, svals


def kaporin(bmat: np.ndarray) -> float:
    """Kaporin number tr(B) / (N det(B)^{1/N}) (Def. 2.3)."""
    n = bmat.shape[0]
    sign, logdet = np.linalg.slogdet(bmat)
    if sign <= 0:
        raise ValueError("Kaporin number needs an SPD matrix")
    return float(np.trace(bmat) / (n * np.exp(logdet / n)))
