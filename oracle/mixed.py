"""Mixed-precision form of the V-cycle (the storage and arithmetic choices of
the FP32/BF16 variant; not in the paper, which works in FP64 throughout).

Storage roundings: A and G are stored in FP32 or BF16, rounded to nearest
with ties to even. BF16 values are obtained by rounding to FP32 first and
then to BF16, the same two steps the storage conversion takes.

The mixed cycle is the V(k,k) cycle of Sec. 5 with every level's A_l and G_l
replaced by their rounded values, FP32 vectors and FP32 arithmetic for the
smoother, the residual and the transfers (the basis change T rounded to FP32
as well), and the exact coarsest-level solve kept in FP64 (FP32 right-hand
side widened, solution rounded back). Each level's bound beta_l is recomputed
by the Lanczos process of Sec. 5 on the rounded operators, evaluated in FP64.
The outer solver is FP64 PCG in its flexible (Polak-Ribiere) form, since the
rounded cycle is not exactly symmetric.

A second form keeps A, the vectors and the arithmetic in FP64 and rounds only
G to BF16 (bf16g_levels): it halves the bytes of the two factor products per
smoothing step while the cycle sees the exact operator.

The FP32 smoother (Algorithm 3 on the rounded A and G, FP32 vectors) and the
two-level mixed V-cycle (FP32 residual and transfers, FP64 coarse Cholesky
fed with FP32 data) are pinned by forward rounding-error bounds around the
exact smoother and cycle on independently rounded operators. The outer
FP64 PCG wrapped around the mixed cycle is not pinned beyond that; its
iteration counts are compared with the FP64 form.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import chebyshev, lanczos
from .bsr import Bsr


def round_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x):
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _bsr32(m: Bsr, vals64) -> sp.bsr_matrix:
    n = m.nb * m.b
    return sp.bsr_matrix((np.asarray(vals64, dtype=np.float32), m.colidx, m.rowptr), shape=(n, n))


@dataclass
class MixedLevel:
    a: sp.bsr_matrix                 # A_l rounded, FP32
    g: sp.bsr_matrix | None = None   # G_l rounded (FP32 or BF16 values), FP32
    gt: sp.bsr_matrix | None = None
    ps: sp.csr_matrix | None = None  # P_s (x) I_b in FP32 (weights exact)
    t: sp.csr_matrix | None = None   # block-diagonal T rounded to FP32, or None
    beta: float = 0.0
    chol: tuple | None = None        # FP64 Cholesky factor of the coarsest A

    def apply_m(self, v):
        return self.gt @ (self.g @ v)

    def restrict(self, r):
        if self.t is not None:
            r = self.t.T @ r
        return self.ps.T @ r

    def prolong(self, xc):
        z = self.ps @ xc
        return self.t @ z if self.t is not None else z


def mixed_levels(levels, g_store: str, starts, iters: int = 100, safety: float = 1.01):
    """Rounded copy of an FP64 oracle hierarchy (oracle.multilevel.Level list).
    g_store: "f32" or "bf16" for G_l; A_l is always FP32. starts[l] is the
    Lanczos start vector of level l."""
    rg = round_bf16 if g_store == "bf16" else round_f32
    out = []
    nl = len(levels)
    for l, lev in enumerate(levels):
        a = lev.a
        if l == nl - 1:
            out.append(MixedLevel(a=_bsr32(a, round_f32(a.vals)), chol=sla.cho_factor(a.dense(), lower=True)))
            continue
        ar = round_f32(a.vals)
        gr = rg(lev.g.vals)
        n = a.nb * a.b
        a64 = sp.bsr_matrix((ar, a.colidx, a.rowptr), shape=(n, n))
        g64 = sp.bsr_matrix((gr, lev.g.colidx, lev.g.rowptr), shape=(n, n))
        gt64 = g64.T.tobsr(blocksize=(a.b, a.b))
        beta, _ = lanczos.lmax(lambda v: g64 @ (a64 @ (gt64 @ v)), np.asarray(starts[l]), iters, safety)
        g32 = _bsr32(lev.g, gr)
        ps = sp.csr_matrix(sp.kron(lev.p_s, sp.identity(a.b), format="csr"), dtype=np.float32)
        t = None
        if lev.basis is not None:
            t = sp.csr_matrix(sp.block_diag([np.asarray(x, dtype=np.float32) for x in round_f32(lev.basis)],
                                            format="csr"), dtype=np.float32)
        out.append(MixedLevel(a=_bsr32(a, ar), g=g32, gt=g32.T.tobsr(blocksize=(a.b, a.b)), ps=ps, t=t,
                              beta=beta))
    return out


def bf16g_levels(levels, starts, iters: int = 100, safety: float = 1.01):
    """The FP64 hierarchy with every smoothed level's G replaced by its BF16
    rounding (A, vectors and arithmetic stay FP64) and beta_l recomputed by
    Lanczos on the rounded factor; the result is used with the plain FP64
    cycle of oracle.multilevel."""
    from .multilevel import Level
    out = []
    for l, lev in enumerate(levels):
        if lev.g is None:
            out.append(lev)
            continue
        g = Bsr(lev.g.rowptr, lev.g.colidx, round_bf16(lev.g.vals), lev.g.b)
        new = Level(a=lev.a, g=g, p_s=lev.p_s, basis=lev.basis).finish()
        new.beta, _ = lanczos.lmax(new.apply_b, np.asarray(starts[l]), iters, safety)
        out.append(new)
    return out


def vcycle_mixed(ml, l: int, b32, k: int):
    """V(k,k) on level l of a mixed hierarchy with zero initial guess; b32 and
    the result are FP32 vectors."""
    lev = ml[l]
    if l == len(ml) - 1:
        return sla.cho_solve(lev.chol, b32.astype(np.float64)).astype(np.float32)
    apply_a = lambda v: lev.a @ v  # noqa: E731
    x = chebyshev.cheb4(apply_a, lev.apply_m, b32, None, lev.beta, k, x_is_zero=True)
    r = b32 - lev.a @ x
    xc = vcycle_mixed(ml, l + 1, lev.restrict(r), k)
    x = x + lev.prolong(xc)
    return chebyshev.cheb4(apply_a, lev.apply_m, b32, x, lev.beta, k)


def precond_mixed(ml, k: int):
    """r (FP64) -> V(k,k) of the mixed hierarchy applied to r rounded to FP32,
    widened back to FP64: the preconditioner of the outer FP64 PCG."""
    return lambda r: vcycle_mixed(ml, 0, r.astype(np.float32), k).astype(np.float64)
