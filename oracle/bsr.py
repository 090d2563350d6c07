"""Block-sparse storage helpers for the oracle (Def. 2.1: block structure).

A block matrix with uniform block size b is held as (rowptr, colidx, vals)
with vals[e] the dense b x b block of entry e. Products use SciPy's BSR
matrix-vector routine as a library primitive.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp


@dataclass
class Bsr:
    rowptr: np.ndarray   # int64, nb + 1
    colidx: np.ndarray   # int32/int64, ascending within each row
    vals: np.ndarray     # (nnzb, b, b) float64
    b: int

    @property
    def nb(self) -> int:
        return len(self.rowptr) - 1

    @property
    def nnzb(self) -> int:
        return len(self.colidx)

    def cols(self, i: int) -> np.ndarray:
        return self.colidx[self.rowptr[i]:self.rowptr[i + 1]]

    def block(self, i: int, j: int) -> np.ndarray:
        """A_ij, or the zero block when (i, j) is outside the pattern."""
        lo, hi = int(self.rowptr[i]), int(self.rowptr[i + 1])
        pos = lo + int(np.searchsorted(self.colidx[lo:hi], j))
        if pos < hi and self.colidx[pos] == j:
            return self.vals[pos]
        return np.zeros((self.b, self.b))

    def sub(self, rows, cols) -> np.ndarray:
        """Dense restriction B[I, J] (Sec. 2, notation after Def. 2.1)."""
        b = self.b
        out = np.zeros((len(rows) * b, len(cols) * b))
        for a, i in enumerate(rows):
            for c, j in enumerate(cols):
                out[a * b:(a + 1) * b, c * b:(c + 1) * b] = self.block(i, j)
        return out

    def scipy(self) -> sp.bsr_matrix:
        n = self.nb * self.b
        return sp.bsr_matrix((self.vals, self.colidx, self.rowptr), shape=(n, n))

    def dense(self) -> np.ndarray:
        return self.scipy().toarray()


def from_problem(p) -> Bsr:
    return Bsr(p.rowptr, p.colidx, p.vals, p.b)


def from_scipy(m, b: int) -> Bsr:
    m = sp.bsr_matrix(m, blocksize=(b, b))
    m.sort_indices()
    return Bsr(m.indptr.astype(np.int64), m.indices.astype(np.int64), np.array(m.data), b)
