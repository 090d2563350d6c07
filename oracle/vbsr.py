"""Block-FSAI with variable block sizes m_i (Def. 2.1 with unequal blocks).

Def. 2.1 partitions the unknowns into blocks of sizes m_1, ..., m_n; every
statement of Def. 2.2 holds for unequal blocks: F_k has m_k rows,
S_kk = (F A F^T)_kk is m_k x m_k and G's block (k, j) is m_k x m_j. This
module is the same literal FP64 implementation as oracle.fsai for that
structure: dense A[P~_k, P~_k]^{-1} per row, S_kk, and G = J F with J the
inverse Cholesky root of S_kk (the reading of S^{-1/2} used throughout).
Products are formed through a scalar SciPy CSR copy of the matrix (a library
primitive). TEST INFRASTRUCTURE ONLY, like the rest of oracle/.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class VBsr:
    rowptr: np.ndarray   # int64, nb + 1
    colidx: np.ndarray   # ascending within each row
    bsize: np.ndarray    # m_i
    vals: np.ndarray     # flat, block e = vals[voff[e]:voff[e+1]] row-major m_i x m_j
    voff: np.ndarray     # nnzb + 1

    @property
    def nb(self) -> int:
        return len(self.rowptr) - 1

    @property
    def boff(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(np.asarray(self.bsize, dtype=np.int64))])

    @property
    def ndof(self) -> int:
        return int(np.sum(self.bsize))

    def cols(self, i: int) -> np.ndarray:
        return self.colidx[self.rowptr[i]:self.rowptr[i + 1]]

    def block(self, i: int, j: int) -> np.ndarray:
        """A_ij (m_i x m_j), or zeros when (i, j) is not stored."""
        lo, hi = int(self.rowptr[i]), int(self.rowptr[i + 1])
        pos = lo + int(np.searchsorted(self.colidx[lo:hi], j))
        mi, mj = int(self.bsize[i]), int(self.bsize[j])
        if pos < hi and self.colidx[pos] == j:
            return self.vals[self.voff[pos]:self.voff[pos + 1]].reshape(mi, mj)
        return np.zeros((mi, mj))

    def sub(self, rows, cols) -> np.ndarray:
        """Dense A[I, J] for block index lists I and J."""
        ro = np.concatenate([[0], np.cumsum([int(self.bsize[i]) for i in rows])]).astype(int)
        co = np.concatenate([[0], np.cumsum([int(self.bsize[j]) for j in cols])]).astype(int)
        out = np.zeros((ro[-1], co[-1]))
        for a, i in enumerate(rows):
            for c, j in enumerate(cols):
                out[ro[a]:ro[a + 1], co[c]:co[c + 1]] = self.block(i, j)
        return out

    def scipy(self) -> sp.csr_matrix:
        """Scalar CSR copy (rows and columns in dof numbering)."""
        boff = self.boff
        r, c, v = [], [], []
        for i in range(self.nb):
            mi = int(self.bsize[i])
            for e in range(self.rowptr[i], self.rowptr[i + 1]):
                j = int(self.colidx[e])
                mj = int(self.bsize[j])
                blk = self.vals[self.voff[e]:self.voff[e + 1]].reshape(mi, mj)
                rr, cc = np.meshgrid(np.arange(mi) + boff[i], np.arange(mj) + boff[j], indexing="ij")
                r.append(rr.ravel())
                c.append(cc.ravel())
                v.append(blk.ravel())
        n = self.ndof
        if not r:
            return sp.csr_matrix((n, n))
        return sp.csr_matrix((np.concatenate(v), (np.concatenate(r), np.concatenate(c))), shape=(n, n))

    def dense(self) -> np.ndarray:
        return self.scipy().toarray()


def from_problem(p) -> VBsr:
    return VBsr(p.rowptr, p.colidx, p.bsize, p.vals, p.voff)


def fsai_row(a: VBsr, k: int, pk):
    """Row k of Def. 2.2 with variable blocks: F[k, P~] = -A[k, P~] A[P~, P~]^{-1},
    S_kk = A_kk - A[k, P~] A[P~, P~]^{-1} A[P~, k], J = L_S^{-1}; returns G's
    blocks on P_k (ascending columns), block j of size m_k x m_j."""
    pt = [int(j) for j in pk if j != k]
    akk = a.block(k, k)
    if pt:
        a_kp = a.sub([k], pt)
        inv_pp = np.linalg.inv(a.sub(pt, pt))
        f_kp = -a_kp @ inv_pp
        s_kk = akk - a_kp @ inv_pp @ a_kp.T
    else:
        f_kp = np.zeros((akk.shape[0], 0))
        s_kk = akk.copy()
    s_kk = 0.5 * (s_kk + s_kk.T)
    jfac = np.linalg.inv(np.linalg.cholesky(s_kk))
    g_kp = jfac @ f_kp
    out, c0 = [], 0
    for j in pt:
        mj = int(a.bsize[j])
        out.append(g_kp[:, c0:c0 + mj])
        c0 += mj
    out.append(jfac)
    return out


def fsai(a: VBsr, prow, pcol) -> VBsr:
    """G = S^{-1/2} F on the pattern, as a variable-block matrix."""
    sizes = []
    for k in range(a.nb):
        for j in pcol[prow[k]:prow[k + 1]]:
            sizes.append(int(a.bsize[k]) * int(a.bsize[int(j)]))
    voff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    vals = np.zeros(int(voff[-1]))
    for k in range(a.nb):
        lo, hi = prow[k], prow[k + 1]
        for e, blk in zip(range(lo, hi), fsai_row(a, k, pcol[lo:hi])):
            vals[voff[e]:voff[e + 1]] = blk.ravel()
    return VBsr(np.asarray(prow, dtype=np.int64), np.asarray(pcol, dtype=np.int64), np.asarray(a.bsize), vals, voff)
