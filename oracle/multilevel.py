"""Galerkin hierarchy, V(k,k)-cycle and preconditioned CG (paper Sec. 5,
opening paragraphs: Galerkin coarse operators A_{l-1} = R_l A_l P_l with
R_l = P_l^T; V(k,k) cycles with fourth-kind Chebyshev smoothing; CG as the
outer solver for symmetric cycles, Sec. 6).

Readings: the coarsest level is solved exactly by a dense Cholesky
factorisation; every level carries its own block-FSAI factor G_l and its own
bound beta_l; the coarse initial guess is zero; PCG stops on the recursive
residual ||r||_2 <= rtol ||b||_2 with x0 = 0.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import chebyshev
from .bsr import Bsr, from_scipy


def block_prolongator(p_s: sp.csr_matrix, b: int, basis=None) -> sp.csr_matrix:
    """P = T (P_s (x) I_b) with T block diagonal (identity when basis is None)."""
    pb = sp.csr_matrix(sp.kron(p_s, sp.identity(b), format="csr"))
    if basis is not None:
        pb = sp.csr_matrix(sp.block_diag(list(basis), format="csr") @ pb)
    return pb


def galerkin(a: Bsr, p_s: sp.csr_matrix, basis=None) -> Bsr:
    """A_c = P^T A P with P = T (P_s (x) I_b), written block by block:

        (A_c)_IJ = sum_i sum_j (P_s)_iI (P_s)_jJ  T_i^T A_ij T_j.

    The congruence T_i^T A_ij T_j is formed for every stored block; the double
    sum with the scalar weights is the same for each of the b*b positions of
    a block, so it is evaluated as the scalar sparse product P_s^T X P_s of
    the matrix X holding that position of every block. The block pattern of
    A_c is the structural product struct(P_s^T struct(A) P_s): blocks that
    cancel to zero stay stored."""
    b = a.b
    nb = a.nb
    rows = np.repeat(np.arange(nb), np.diff(a.rowptr))
    cols = np.asarray(a.colidx, dtype=np.int64)
    vals = np.asarray(a.vals, dtype=np.float64)
    if basis is not None:
        t = np.asarray(basis, dtype=np.float64)
        cong = np.empty_like(vals)
        step = 1 << 18
        for s0 in range(0, len(cols), step):
            s1 = min(s0 + step, len(cols))
            cong[s0:s1] = np.swapaxes(t[rows[s0:s1]], 1, 2) @ vals[s0:s1] @ t[cols[s0:s1]]
        vals = cong
    ps = sp.csr_matrix(p_s, dtype=np.float64)
    nc = ps.shape[1]
    ones_a = sp.csr_matrix((np.ones(len(cols)), cols, a.rowptr), shape=(nb, nb))
    ones_p = sp.csr_matrix((np.ones(ps.nnz), ps.indices, ps.indptr), shape=ps.shape)
    struct = sp.csr_matrix(ones_p.T @ ones_a @ ones_p)
    struct.sort_indices()
    srows = np.repeat(np.arange(nc, dtype=np.int64), np.diff(struct.indptr))
    key = srows * nc + struct.indices
    out = np.zeros((struct.nnz, b, b))
    for r in range(b):
        for c in range(b):
            x = sp.csr_matrix((vals[:, r, c], cols, a.rowptr), shape=(nb, nb))
            prod = sp.coo_matrix(ps.T @ x @ ps)
            pos = np.searchsorted(key, prod.row.astype(np.int64) * nc + prod.col)
            out[pos, r, c] = prod.data
    return Bsr(struct.indptr.astype(np.int64), struct.indices.astype(np.int64), out, b)


@dataclass
class Level:
    a: Bsr
    g: Bsr | None = None          # block-FSAI factor (None on the coarsest level)
    beta: float = 0.0
    p_s: sp.csr_matrix | None = None   # prolongation from level l+1 to level l
    basis: np.ndarray | None = None    # block-diagonal T of P = T (P_s (x) I_b)
    chol: tuple | None = None
    a_sp: sp.bsr_matrix = field(default=None, repr=False)
    g1: Bsr | None = None         # inner factor of nested FSAI (Sec. 2.2), or None
    g_sp: sp.bsr_matrix = field(default=None, repr=False)
    gt_sp: sp.bsr_matrix = field(default=None, repr=False)
    g1_sp: sp.bsr_matrix = field(default=None, repr=False)
    g1t_sp: sp.bsr_matrix = field(default=None, repr=False)
    pb: sp.csr_matrix = field(default=None, repr=False)

    def finish(self):
        self.a_sp = self.a.scipy()
        if self.g is not None:
            self.g_sp = self.g.scipy()
            self.gt_sp = self.g_sp.T.tobsr(blocksize=(self.a.b, self.a.b))
        if self.g1 is not None:
            self.g1_sp = self.g1.scipy()
            self.g1t_sp = self.g1_sp.T.tobsr(blocksize=(self.a.b, self.a.b))
        if self.p_s is not None:
            self.pb = block_prolongator(self.p_s, self.a.b, self.basis)
        return self

    def apply_a(self, v):
        return self.a_sp @ v

    def apply_m(self, v):
        if self.g1 is not None:
            return self.gt_sp @ (self.g1t_sp @ (self.g1_sp @ (self.g_sp @ v)))
        return self.gt_sp @ (self.g_sp @ v)

    def apply_b(self, v):
        """v -> G^ A G^T v with G^ = G (or G1 G0 when nested): the operator
        whose largest eigenvalue bounds the spectrum of M A."""
        if self.g1 is not None:
            return self.g1_sp @ (self.g_sp @ (self.a_sp @ (self.gt_sp @ (self.g1t_sp @ v))))
        return self.g_sp @ (self.a_sp @ (self.gt_sp @ v))


def coarse_factor(a: Bsr):
    return sla.cho_factor(a.dense(), lower=True)


def smooth(lev: Level, b, x, degree: int, smoother: str = "cheb4", param: float = 0.0, x_is_zero=False):
    """One smoother application on a level: "cheb4" (Algorithm 3 on
    [0, beta]), "cheb1" (Algorithm 2 on [param * beta, beta]) or
    "richardson" (omega = param)."""
    if smoother == "cheb4":
        return chebyshev.cheb4(lev.apply_a, lev.apply_m, b, x, lev.beta, degree, x_is_zero=x_is_zero)
    if smoother == "cheb1":
        return chebyshev.cheb1(lev.apply_a, lev.apply_m, b, x, param * lev.beta, lev.beta, degree,
                               x_is_zero=x_is_zero)
    if smoother == "richardson":
        return chebyshev.richardson(lev.apply_a, lev.apply_m, b, x, param, degree, x_is_zero=x_is_zero)
    raise ValueError(smoother)


def vcycle(levels: list[Level], l: int, b, k: int, smoother: str = "cheb4", param: float = 0.0,
           cycle: str = "vkk"):
    """V(k,k) with zero initial guess: pre-smooth, residual, restrict,
    recurse, prolongate, post-smooth; exact solve on the coarsest level.
    cycle="v2k0": Sec. 5's non-symmetric V(2k,0), one pre-smoothing
    application of degree 2k and no post-smoothing."""
    lev = levels[l]
    if l == len(levels) - 1:
        return sla.cho_solve(lev.chol, b)
    pre = 2 * k if cycle == "v2k0" else k
    x = smooth(lev, b, None, pre, smoother, param, x_is_zero=True)
    r = b - lev.apply_a(x)
    xc = vcycle(levels, l + 1, lev.pb.T @ r, k, smoother, param, cycle)
    x = x + lev.pb @ xc
    if cycle == "v2k0":
        return x
    return smooth(lev, b, x, k, smoother, param)


def vcycle_x(levels: list[Level], b, x, k: int, smoother: str = "cheb4", param: float = 0.0, cycle: str = "vkk"):
    """One cycle from a given initial guess x on level 0."""
    lev = levels[0]
    if len(levels) == 1:
        return sla.cho_solve(lev.chol, b)
    x = smooth(lev, b, x, 2 * k if cycle == "v2k0" else k, smoother, param)
    r = b - lev.apply_a(x)
    xc = vcycle(levels, 1, lev.pb.T @ r, k, smoother, param, cycle)
    x = x + lev.pb @ xc
    if cycle == "v2k0":
        return x
    return smooth(lev, b, x, k, smoother, param)


def pcg(apply_a, apply_prec, b, rtol: float, maxit: int, flexible: bool = False):
    """Preconditioned CG from x0 = 0. Fletcher-Reeves beta, or Polak-Ribiere
    (z, r - r_old)/(r_old, z_old) when flexible. Returns
    (x, iterations, recursive residual history, true relative residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = float(np.linalg.norm(b))
    hist = [float(np.linalg.norm(r)) / bnorm]
    if hist[0] <= rtol:
        return x, 0, hist, hist[0]
    z = apply_prec(r)
    p = z.copy()
    rz = float(r @ z)
    it = 0
    for it in range(1, maxit + 1):
        q = apply_a(p)
        pq = float(p @ q)
        if pq <= 0:
            raise ArithmeticError("PCG breakdown: p^T A p <= 0")
        alpha = rz / pq
        x = x + alpha * p
        r_old = r
        r = r - alpha * q
        hist.append(float(np.linalg.norm(r)) / bnorm)
        if hist[-1] <= rtol:
            break
        z = apply_prec(r)
        rz_new = float(r @ z)
        betac = (float(z @ (r - r_old)) if flexible else rz_new) / rz
        rz = rz_new
        p = z + betac * p
    true_res = float(np.linalg.norm(b - apply_a(x))) / bnorm
    return x, it, hist, true_res


def bicgstab(apply_a, apply_prec, b, rtol: float, maxit: int):
    """Right-preconditioned BiCGStab (van der Vorst, 1992) from x0 = 0 with
    shadow residual r^ = b: the outer solver that accepts the non-symmetric
    V(2k,0) preconditioner (Sec. 6). Stops when the recursive residual
    (also checked at the half step s) satisfies ||r|| <= rtol ||b||. Returns
    (x, iterations, residual history per half step, true relative residual)."""
    x = np.zeros_like(b)
    r = b.copy()
    rhat = b.copy()
    bnorm = float(np.linalg.norm(b))
    hist = [float(np.linalg.norm(r)) / bnorm]
    if hist[0] <= rtol:
        return x, 0, hist, hist[0]
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    rho_old = alpha = omega = 1.0
    it = 0
    for it in range(1, maxit + 1):
        rho = float(rhat @ r)
        if rho == 0.0:
            raise ArithmeticError("BiCGStab breakdown: (r^, r) = 0")
        if it == 1:
            p = r.copy()
        else:
            p = r + (rho / rho_old) * (alpha / omega) * (p - omega * v)
        ph = apply_prec(p)
        v = apply_a(ph)
        alpha = rho / float(rhat @ v)
        s = r - alpha * v
        hist.append(float(np.linalg.norm(s)) / bnorm)
        if hist[-1] <= rtol:
            x = x + alpha * ph
            break
        sh = apply_prec(s)
        t = apply_a(sh)
        omega = float(t @ s) / float(t @ t)
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        hist.append(float(np.linalg.norm(r)) / bnorm)
        if hist[-1] <= rtol:
            break
        rho_old = rho
    true_res = float(np.linalg.norm(b - apply_a(x))) / bnorm
    return x, it, hist, true_res


def energy_factor(levels: list[Level], e0, k: int, tol: float = 1e-8, maxit: int = 50, smoother: str = "cheb4",
                  param: float = 0.0, cycle: str = "vkk"):
    """Convergence factor in the energy norm (Example 5.1's protocol with b = 0):
    iterate e <- V(0, e) until ||e||_A < tol ||e0||_A or maxit cycles, and
    return (||e_n||_A^2 / ||e_0||_A^2)^{1/(2n)} and n."""
    a0 = levels[0]
    e = np.array(e0, dtype=np.float64)
    en0 = float(e @ a0.apply_a(e))
    zero = np.zeros_like(e)
    n = 0
    en = en0
    while n < maxit:
        e = vcycle_x(levels, zero, e, k, smoother, param, cycle)
        n += 1
        en = float(e @ a0.apply_a(e))
        if np.sqrt(en / en0) < tol:
            break
    return (en / en0) ** (1.0 / (2 * n)), n
