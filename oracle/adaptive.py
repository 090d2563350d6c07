"""Adaptive block-FSAI pattern (Algorithm 1, Sec. 2.1, with Lemma 2.4).

Block rows evolve independently: in every adaptive step, row k of F depends
only on A and on P_k (Eq. fsai_f_definition), and so do H_kc = (FA)_kc and
W_c. The oracle therefore runs Algorithm 1 one row at a time; the result is
the same pattern as running all rows in lock step.

Readings (see the package docstring): 0-based indices, candidates c < k,
structural candidate set, tie window 1e-9 on g = -log rho, smallest index
among ties, add when g* > -log(tau) + GAIN_EPS.
"""
from __future__ import annotations

import math

import numpy as np

from .bsr import Bsr

TIE_REL = 1e-9
GAIN_EPS = 1e-12


def _logdet_spd(m: np.ndarray) -> float:
    sign, val = np.linalg.slogdet(m)
    if sign <= 0:
        raise np.linalg.LinAlgError("matrix not positive definite in Algorithm 1")
    return float(val)


def candidates(a: Bsr, k: int, pk) -> list[int]:
    """C = {c < k : H_kc not identically zero} read structurally.

    The block pattern of row k of H = F A is the union of the patterns of the
    rows A_j with j in P_k; entries already in P_k are zero by Eq. fsai_helper.
    """
    pset = set(int(j) for j in pk)
    cand = set()
    for j in pset:
        for c in a.cols(j):
            c = int(c)
            if c < k and c not in pset:
                cand.add(c)
    return sorted(cand)


def logdet_one_minus(c: np.ndarray) -> float:
    """log det(I - C) for SPD C with ||C|| < 1, by a Cholesky factorisation of
    I - C whose pivots are formed as 1 - s_i and logged with log1p(-s_i), so
    that small C keep their relative accuracy."""
    m = c.shape[0]
    lo = np.zeros((m, m))
    out = 0.0
    for i in range(m):
        for j in range(i):
            lo[i, j] = (-c[i, j] - lo[i, :j] @ lo[j, :j]) / lo[j, j]
        s = c[i, i] + lo[i, :i] @ lo[i, :i]
        if s >= 1.0:
            raise np.linalg.LinAlgError("rho_c <= 0 in Algorithm 1")
        lo[i, i] = np.sqrt(1.0 - s)
        out += np.log1p(-s)
    return out


def gains(a: Bsr, k: int, pk, cand):
    """g_c = -log rho_c for each candidate (Lemma 2.4 and Algorithm 1).

    rho_c = det(W_c - H_kc^T H_kk^{-1} H_kc) / det(W_c), with
    H_kk = A_kk - A[k,P~] A[P~,P~]^{-1} A[P~,k]       (= (FAF^T)_kk, Lemma 2.1)
    H_kc = A_kc - A[k,P~] A[P~,P~]^{-1} A[P~,c]       (= (FA)_kc)
    W_c  = A_cc - A[c,P~] A[P~,P~]^{-1} A[P~,c].
    The ratio is evaluated as det(I - X X^T) with X = L_W^{-1} H_kc^T L_H^{-T}
    (W_c = L_W L_W^T, H_kk = L_H L_H^T): the same number, obtained by taking
    det(W_c) out of the numerator, but free of the cancellation of two large
    log-determinants when the gain is small.
    """
    pt = [int(j) for j in pk if j != k]
    akk = a.block(k, k)
    if pt:
        inv_pp = np.linalg.inv(a.sub(pt, pt))
        a_kp = a.sub([k], pt)
    h_kk = akk - (a_kp @ inv_pp @ a_kp.T if pt else 0.0)
    l_h = np.linalg.cholesky(0.5 * (h_kk + h_kk.T))
    out = []
    for c in cand:
        a_kc = a.block(k, c)
        a_cc = a.block(c, c)
        if pt:
            a_pc = a.sub(pt, [c])
            h_kc = a_kc - a_kp @ inv_pp @ a_pc
            w_c = a_cc - a_pc.T @ inv_pp @ a_pc
        else:
            h_kc = a_kc
            w_c = a_cc
        l_w = np.linalg.cholesky(0.5 * (w_c + w_c.T))
        x = np.linalg.solve(l_w, np.linalg.solve(l_h, h_kc).T)
        out.append(-logdet_one_minus(x @ x.T))
    return np.array(out)


def gains_logdet(a: Bsr, k: int, pk, cand):
    """The same g_c taken literally as log det(W_c) - log det(W_c - H_kc^T
    H_kk^{-1} H_kc); agrees with ``gains`` up to the cancellation error."""
    pt = [int(j) for j in pk if j != k]
    akk = a.block(k, k)
    if pt:
        inv_pp = np.linalg.inv(a.sub(pt, pt))
        a_kp = a.sub([k], pt)
    h_kk = akk - (a_kp @ inv_pp @ a_kp.T if pt else 0.0)
    h_kk_inv = np.linalg.inv(h_kk)
    out = []
    for c in cand:
        a_kc = a.block(k, c)
        a_cc = a.block(c, c)
        if pt:
            a_pc = a.sub(pt, [c])
            h_kc = a_kc - a_kp @ inv_pp @ a_pc
            w_c = a_cc - a_pc.T @ inv_pp @ a_pc
        else:
            h_kc = a_kc
            w_c = a_cc
        out.append(_logdet_spd(w_c) - _logdet_spd(w_c - h_kc.T @ h_kk_inv @ h_kc))
    return np.array(out)


def pick(cand, g, tie_rel: float = TIE_REL):
    """Tie rule: among gains within a relative window of the best, the
    smallest block index. Returns (c*, g*, smallest non-tied gap)."""
    gmax = float(np.max(g))
    thresh = gmax - tie_rel * abs(gmax)
    tied = [c for c, gc in zip(cand, g) if gc >= thresh]
    others = [gmax - gc for gc in g if gc < thresh]
    gap = min(others) / abs(gmax) if others and gmax != 0 else math.inf
    return min(tied), gmax, gap


def adaptive_row(a: Bsr, k: int, tmax: int, tau: float = 1.0, p0=None,
                 tie_rel: float = TIE_REL, gain_eps: float = GAIN_EPS):
    """Final P_k of Algorithm 1 for one row; P0 defaults to the diagonal."""
    pk = sorted(set([k] if p0 is None else [int(j) for j in p0]) | {k})
    thresh = -math.log(tau) + gain_eps
    for _ in range(tmax):
        cand = candidates(a, k, pk)
        if not cand:
            break
        g = gains(a, k, pk, cand)
        cstar, gstar, _ = pick(cand, g, tie_rel)
        if gstar > thresh:          # rho_{c*} < tau
            pk = sorted(pk + [cstar])
        else:
            break
    return pk


def adaptive_pattern(a: Bsr, tmax: int, tau: float = 1.0, rows=None, p0_pattern=None, **kw):
    """Algorithm 1 for all rows (or the listed ones): CSR of final patterns.
    p0_pattern: the initial pattern P0 as CSR (prow, pcol); None = diagonal."""
    rows = range(a.nb) if rows is None else rows
    prow, pcol = [0], []
    for k in rows:
        k = int(k)
        p0 = None if p0_pattern is None else p0_pattern[1][p0_pattern[0][k]:p0_pattern[0][k + 1]]
        pcol.extend(adaptive_row(a, k, tmax, tau, p0=p0, **kw))
        prow.append(len(pcol))
    return np.array(prow, dtype=np.int64), np.array(pcol, dtype=np.int64)
