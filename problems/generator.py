"""Synthetic PUM-shaped block-sparse SPD matrices.

Shape of the workloads (paper, Sec. 4 and Sec. 5): a patch grid of 2^l
patches per side in d dimensions (Fig. pum_cover), one dense local block of
size b = C(p+d, d) per patch, block couplings between overlapping patches, and
SPD operators of biharmonic (fourth order) or triharmonic (sixth order) type.
The PUM assembly itself is not reproduced; instead

    A = R^T (D (x) I_b) R,   D = L^q,

with L the unscaled Dirichlet Laplacian on the patch grid (2d on the
diagonal, -1 for each grid neighbour), q = 2 (biharmonic-like) or 3
(triharmonic-like), and R block-diagonal with R_i = Q_i diag(exp(u_i)),
Q_i Haar-orthogonal and u_i ~ U[-1, 1]^b. Block (i, j) of A is
D_ij R_i^T R_j. Blocks are numbered lexicographically with x fastest:
i = ix + n*iy (+ n^2*iz).

Random streams: SeedSequence(seed).spawn(4) gives, in order, the streams for
Q, for u, for right-hand sides and for Lanczos start vectors.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import comb

import numpy as np
import scipy.sparse as sp

STREAM_Q, STREAM_U, STREAM_RHS, STREAM_LANCZOS = range(4)


def _streams(seed: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(4)]


def grid_sizes(n: int, levels: int) -> list[int]:
    """Patches per side on each level, finest first (n, n/2, ...)."""
    out = []
    for _ in range(levels):
        out.append(n)
        n //= 2
    return out


def laplacian(n: int, dim: int) -> sp.csr_matrix:
    """Unscaled Dirichlet Laplacian on an n^dim patch grid, x fastest.

    Integer valued: 2*dim on the diagonal and -1 for each of the (up to)
    2*dim grid neighbours. Exact in floating point.
    """
    one = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    eye = sp.identity(n, format="csr")
    if dim == 1:
        return one.astype(np.float64)
    if dim == 2:
        lap = sp.kron(eye, one) + sp.kron(one, eye)
    elif dim == 3:
        lap = (sp.kron(eye, sp.kron(eye, one)) + sp.kron(eye, sp.kron(one, eye))
               + sp.kron(one, sp.kron(eye, eye)))
    else:
        raise ValueError("dim must be 1, 2 or 3")
    return sp.csr_matrix(lap, dtype=np.float64)


def stencil_matrix(n: int, dim: int, power: int) -> sp.csr_matrix:
    """D = L^power on the patch grid, with sorted column indices."""
    lap = laplacian(n, dim)
    d = lap
    for _ in range(power - 1):
        d = d @ lap
    d = sp.csr_matrix(d)
    d.eliminate_zeros()
    d.sort_indices()
    return d


def _haar_orthogonal(rng: np.random.Generator, count: int, b: int) -> np.ndarray:
    """Haar-distributed orthogonal b x b matrices: QR of a Gaussian matrix
    with the signs of R's diagonal moved into Q (Mezzadri's correction)."""
    z = rng.standard_normal((count, b, b))
    q, r = np.linalg.qr(z)
    sgn = np.sign(np.einsum("kii->ki", r))
    sgn[sgn == 0] = 1.0
    return q * sgn[:, None, :]


@dataclass
class Problem:
    """A block-sparse SPD matrix in BSR form plus the data that made it."""

    n: int                 # patches per side
    dim: int
    b: int                 # block size
    power: int             # D = L^power
    seed: int
    rowptr: np.ndarray     # int64, nb+1
    colidx: np.ndarray     # int32, nnzb (ascending within each row)
    vals: np.ndarray       # float64, (nnzb, b, b), each block row-major
    dstencil: sp.csr_matrix = field(repr=False)  # the scalar D
    rfac: np.ndarray = field(repr=False)         # (nb, b, b) block-diagonal R
    rinv: np.ndarray = field(repr=False)         # (nb, b, b) R^{-1} = diag(exp(-u)) Q^T

    @property
    def nb(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnzb(self) -> int:
        return int(self.colidx.shape[0])

    @property
    def ndof(self) -> int:
        return self.nb * self.b

    def to_scipy(self) -> sp.bsr_matrix:
        return sp.bsr_matrix((self.vals, self.colidx, self.rowptr),
                             shape=(self.ndof, self.ndof))


def make_problem(n: int, dim: int, b: int, power: int, seed: int = 0,
                 rotate: bool = True, chunk: int = 1 << 19) -> Problem:
    """Build A = R^T (D (x) I_b) R on an n^dim patch grid.

    With rotate=False, R = I and A = D (x) I_b (the scalar problem repeated
    per block component).
    """
    dmat = stencil_matrix(n, dim, power)
    nb = dmat.shape[0]
    streams = _streams(seed)
    if rotate:
        q = _haar_orthogonal(streams[STREAM_Q], nb, b)
        u = streams[STREAM_U].uniform(-1.0, 1.0, size=(nb, b))
        rfac = q * np.exp(u)[:, None, :]          # Q_i diag(exp u_i)
        rinv = np.swapaxes(q, 1, 2) * np.exp(-u)[:, :, None]
    else:
        rfac = np.broadcast_to(np.eye(b), (nb, b, b)).copy()
        rinv = rfac.copy()
    rowptr = dmat.indptr.astype(np.int64)
    colidx = dmat.indices.astype(np.int32)
    rows = np.repeat(np.arange(nb, dtype=np.int64), np.diff(rowptr))
    dval = dmat.data
    vals = np.empty((colidx.shape[0], b, b), dtype=np.float64)
    for s in range(0, colidx.shape[0], chunk):
        e = min(s + chunk, colidx.shape[0])
        ri = rfac[rows[s:e]]
        rj = rfac[colidx[s:e]]
        # D_ij * R_i^T R_j
        np.matmul(np.swapaxes(ri, 1, 2), rj, out=vals[s:e])
        vals[s:e] *= dval[s:e, None, None]
    return Problem(n=n, dim=dim, b=b, power=power, seed=seed, rowptr=rowptr,
                   colidx=colidx, vals=vals, dstencil=dmat, rfac=rfac, rinv=rinv)


@dataclass
class VarProblem:
    """Block-sparse SPD matrix with variable block sizes m_i (Def. 2.1's block
    structure with unequal blocks). Block e = (i, j) is the m_i x m_j array
    vals[voff[e]:voff[e+1]] in row-major order."""

    n: int
    dim: int
    power: int
    seed: int
    bsize: np.ndarray      # int32, nb: m_i
    rowptr: np.ndarray     # int64, nb+1
    colidx: np.ndarray     # int32, nnzb (ascending within each row)
    vals: np.ndarray       # float64, sum over stored blocks of m_i m_j
    voff: np.ndarray       # int64, nnzb+1
    dstencil: sp.csr_matrix = field(repr=False)

    @property
    def nb(self) -> int:
        return int(self.rowptr.shape[0] - 1)

    @property
    def nnzb(self) -> int:
        return int(self.colidx.shape[0])

    @property
    def boff(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.bsize.astype(np.int64))])

    @property
    def ndof(self) -> int:
        return int(self.bsize.sum())


def vb_block_sizes(n: int, dim: int, p_interior: int, p_boundary: int) -> np.ndarray:
    """Local space sizes C(p + d, d) per patch of an n^dim grid: polynomial
    degree p_boundary on the patches that touch the boundary (any coordinate 0
    or n - 1), p_interior elsewhere; x fastest."""
    coords = np.indices((n,) * dim).reshape(dim, -1)[::-1]
    boundary = np.any((coords == 0) | (coords == n - 1), axis=0)
    return np.where(boundary, pum_block_size(p_boundary, dim), pum_block_size(p_interior, dim)).astype(np.int32)


def make_vb_problem(n: int, dim: int, power: int, p_interior: int = 2, p_boundary: int = 3,
                    seed: int = 0) -> VarProblem:
    """A = B^T (D (x) I_M) B on an n^dim patch grid with block sizes m_i from
    vb_block_sizes, M = max m_i: B is block diagonal with the M x m_i blocks
    B_i = Q_i[:, :m_i] diag(exp(u_i)), Q_i Haar-orthogonal M x M and
    u_i ~ U[-1, 1]^{m_i}, so block (i, j) is D_ij B_i^T B_j (m_i x m_j) and
    A_ii = D_ii diag(exp(2 u_i)). A is SPD because B has full column rank.
    Streams as in make_problem: SeedSequence(seed).spawn(4) -> (Q, u, RHS,
    Lanczos)."""
    dmat = stencil_matrix(n, dim, power)
    nb = dmat.shape[0]
    m = vb_block_sizes(n, dim, p_interior, p_boundary)
    big = int(m.max())
    streams = _streams(seed)
    q = _haar_orthogonal(streams[STREAM_Q], nb, big)
    u = streams[STREAM_U].uniform(-1.0, 1.0, size=(nb, big))
    rowptr = dmat.indptr.astype(np.int64)
    colidx = dmat.indices.astype(np.int32)
    rows = np.repeat(np.arange(nb, dtype=np.int64), np.diff(rowptr))
    sizes = m[rows].astype(np.int64) * m[colidx]
    voff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    vals = np.empty(int(voff[-1]))
    bfull = q * np.exp(u)[:, None, :]          # Q_i diag(exp u_i); B_i is its first m_i columns
    mi, mj = m[rows], m[colidx]
    for a in np.unique(m):
        for c in np.unique(m):
            sel = np.nonzero((mi == a) & (mj == c))[0]
            for s0 in range(0, len(sel), 1 << 16):
                es = sel[s0:s0 + (1 << 16)]
                blk = np.swapaxes(bfull[rows[es], :, :a], 1, 2) @ bfull[colidx[es], :, :c]
                blk *= dmat.data[es, None, None]
                idx = voff[es][:, None] + np.arange(a * c)[None, :]
                vals[idx] = blk.reshape(len(es), -1)
    return VarProblem(n=n, dim=dim, power=power, seed=seed, bsize=m, rowptr=rowptr, colidx=colidx, vals=vals,
                      voff=voff, dstencil=dmat)


def pum_block_size(p: int, dim: int) -> int:
    """dim V_i = C(p + d, d) for local polynomials of degree p."""
    return comb(p + dim, dim)


def _lagrange_weights(nodes, t):
    out = []
    for i, xi in enumerate(nodes):
        w = 1.0
        for j, xj in enumerate(nodes):
            if j != i:
                w *= (t - xj) / (xi - xj)
        out.append(w)
    return out


def prolongator_1d(nc: int, order: int = 2, boundary: str = "dirichlet") -> sp.csr_matrix:
    """Cell-centred 1D interpolation from nc to 2*nc cells.

    In coarse units, fine cell 2I+a sits at t = I - 1/4 (a = 0) or I + 1/4
    (a = 1). The unscaled Dirichlet Laplacian on the fine grid vanishes half a
    fine cell beyond its outer cells, i.e. at the coarse coordinates -3/4 and
    nc - 1/4.

    boundary="dirichlet": the fine value is the Lagrange interpolant through
    the `order` points nearest to t among the coarse cells and these two
    boundary points (value 0 there); order 2 is linear (weights 3/4, 1/4 in
    the interior, 2/3 next to the boundary), order 4 is cubic (interior
    weights (-5, 35, 105, -7)/128 on I-2..I+1 for a = 0, mirrored for a = 1),
    exact for polynomials of degree order-1 that vanish at the boundary.
    boundary="zero_ghost" (order 2 only): 3/4 of cell I and 1/4 of its
    neighbour on the same side, a neighbour outside the grid dropped.
    """
    nf = 2 * nc
    rows, cols, vals = [], [], []
    if boundary == "zero_ghost":
        if order != 2:
            raise ValueError("zero_ghost is defined for order 2 only")
        for f in range(nf):
            big, a = divmod(f, 2)
            rows.append(f)
            cols.append(big)
            vals.append(0.75)
            other = big - 1 if a == 0 else big + 1
            if 0 <= other < nc:
                rows.append(f)
                cols.append(other)
                vals.append(0.25)
        return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))
    if boundary != "dirichlet":
        raise ValueError(boundary)
    if order < 1 or order > nc + 2:
        raise ValueError("bad interpolation order")
    lo, hi = -0.75, nc - 0.25
    for f in range(nf):
        big, a = divmod(f, 2)
        t = big - 0.25 if a == 0 else big + 0.25
        # the order nearest points; no two candidates are equally far from t
        near = sorted(range(-1, nc + 1), key=lambda i: abs((lo if i < 0 else hi if i >= nc else i) - t))[:order]
        nodes = sorted(lo if i < 0 else hi if i >= nc else float(i) for i in near)
        for x, w in zip(nodes, _lagrange_weights(nodes, t)):
            if x in (lo, hi):
                continue
            rows.append(f)
            cols.append(int(x))
            vals.append(w)
    m = sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))
    m.sort_indices()
    return m


def prolongator(nc: int, dim: int, order: int = 2, boundary: str = "dirichlet") -> sp.csr_matrix:
    """Tensor-product patch prolongator P_s from nc^dim to (2nc)^dim patches
    (scalar weights; the block operator is P_s (x) I_b). x is fastest."""
    p1 = prolongator_1d(nc, order, boundary)
    p = p1
    for _ in range(dim - 1):
        p = sp.kron(p1, p)
    p = sp.csr_matrix(p)
    p.sort_indices()
    return p


def level_basis(p: Problem, levels: int) -> list:
    """Block-diagonal basis change of each level's prolongation.

    The patch prolongator P_s (x) I_b interpolates the coefficients of the
    unrotated local bases; the finest level's local bases are rotated by R
    (A = R^T (D (x) I_b) R), so its prolongation is R^{-1} (P_s (x) I_b). The
    Galerkin coarse operators carry no rotation (identity, None). Entry l
    belongs to the prolongation from level l+1 to level l.
    """
    return [p.rinv if l == 0 else None for l in range(levels - 1)]


def rhs(seed: int, ndof: int) -> np.ndarray:
    """Right-hand side ~ N(0, 1)^ndof from the seed's RHS stream."""
    return _streams(seed)[STREAM_RHS].standard_normal(ndof)


def lanczos_starts(seed: int, sizes: list[int]) -> list[np.ndarray]:
    """One N(0,1) start vector per level, drawn in level order from the
    seed's Lanczos stream."""
    rng = _streams(seed)[STREAM_LANCZOS]
    return [rng.standard_normal(m) for m in sizes]


def uniform_start(seed: int, ndof: int) -> np.ndarray:
    """Initial error with entries in U(-1, 1) for convergence-factor runs."""
    return np.random.default_rng(np.random.SeedSequence([seed, 7919])).uniform(-1.0, 1.0, ndof)


def mlp_init(seed: int) -> np.ndarray:
    """He-uniform initial weights (zero biases) for the 6-64-64-1 network,
    in the layout W1[64][6], b1[64], W2[64][64], b2[64], W3[64], b3."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 4673]))
    w1 = rng.uniform(-1, 1, (64, 6)) * np.sqrt(6.0 / 6)
    w2 = rng.uniform(-1, 1, (64, 64)) * np.sqrt(6.0 / 64)
    w3 = rng.uniform(-1, 1, 64) * np.sqrt(6.0 / 64)
    return np.concatenate([w1.ravel(), np.zeros(64), w2.ravel(), np.zeros(64), w3, [0.0]]).astype(np.float32)


def permutation(seed: int, n: int) -> np.ndarray:
    """Seeded random permutation of n training rows."""
    return np.random.default_rng(np.random.SeedSequence([seed, 271828])).permutation(n).astype(np.int64)
