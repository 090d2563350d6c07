"""Pin for the mixed-precision smoother of the oracle (FP32 storage of A and
G, G optionally BF16, FP32 vectors and arithmetic; Algorithm 3 inside the
cycle of Sec. 5).

The exact smoother on the rounded operators is known up to FP64 rounding, so
the FP32 evaluation must lie within a rigorous forward rounding-error bound
of it. The bound follows each vector of the recurrence with the standard
model fl(a op b) = (a op b)(1 + e), |e| <= u, and the bound
|fl(A v) - A v| <= gamma_n |A| |v| for a sum of n products, gamma_n =
n u / (1 - n u) (Higham, Accuracy and Stability of Numerical Algorithms,
Sec. 3.1): with x, delta, r the exact iterates and x^, delta^, r^ the
computed ones,
    |r^ - r|      <= |A| e_x + gamma_nA |A||x^| + gamma_1 |r^|,
    |t^ - G r|    <= |G| e_r + gamma_nG |G||r^|,
    |z^ - G^T t|  <= |G^T| e_t + gamma_nGt |G^T||t^|,
    |delta^ - delta| <= |c| e_delta + |s| e_z + gamma_4 (|c||delta^_prev| + |s||z^|),
    |x^ - x|      <= e_x + e_delta + gamma_1 |x^|,
where c, s are the increment coefficients of Algorithm 3 (each rounded once
to the working precision). The same bound with the FP64 unit roundoff covers
the FP64 evaluation, so the two evaluations differ by at most the sum.

The reference operators are rounded with torch's CPU conversions, not with
the oracle's rounding functions, so the pin also checks which rounding each
operator received: the BF16-G smoother is compared with the FP32-G exact
smoother too, and must fall outside the bound there.
"""
import functools

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import chebyshev, mixed, solver
from oracle.bsr import from_problem
from problems import grid_sizes, lanczos_starts, make_problem, prolongator, rhs

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def _gamma(n, u):
    return n * u / (1.0 - n * u)


def _round_torch(vals, store):
    import torch
    t = torch.from_numpy(np.asarray(vals, dtype=np.float64))
    dt = torch.bfloat16 if store == "bf16" else torch.float32
    return t.to(torch.float32).to(dt).to(torch.float64).numpy()


def _max_row_terms(m):
    return int(np.diff(sp.csr_matrix(m).indptr).max())


def _run(a, g, gt, b, x0, beta, k, dtype):
    """Runs the oracle's Algorithm 3 with operators a, g, gt (SciPy sparse of
    `dtype`) and records what it passes through the operator callbacks."""
    xs, ys, rs, ts, zs = [], [], [], [], []

    def apply_a(v):
        xs.append(np.asarray(v, dtype=np.float64).copy())
        y = a @ v
        ys.append(np.asarray(y, dtype=np.float64).copy())
        return y

    def apply_m(v):
        rs.append(np.asarray(v, dtype=np.float64).copy())
        t = g @ v
        ts.append(np.asarray(t, dtype=np.float64).copy())
        z = gt @ t
        zs.append(np.asarray(z, dtype=np.float64).copy())
        return z

    bb = np.asarray(b, dtype=dtype)
    xz = x0 is None
    x = chebyshev.cheb4(apply_a, apply_m, bb, None if xz else np.asarray(x0, dtype=dtype), beta, k, x_is_zero=xz)
    return np.asarray(x, dtype=np.float64), xs, rs, ts, zs


def _bound(a, g, gt, x0, beta, k, rec, u):
    """2-norm bound on x^ - x for one recorded evaluation.

    Each step's rounding errors are bounded componentwise from the computed
    vectors (the model in the module docstring); they enter the exact error
    recurrence of the increment form,
        E_d,i = c_i E_d,i-1 - s_i M A E_x,i-1 + u_i,
        E_x,i = E_x,i-1 + E_d,i + f_x,i,
    with u_i = s_i (G^T G f_r + G^T f_t + f_z) + f_delta, and are carried to
    the result by the products of the exact transition matrices, whose
    2-norms are computed densely (small n). The factor 1.01 covers terms of
    second order in u and the FP64 evaluation of the bound itself.
    """
    x_out, xs, rs, ts, zs = rec
    ad, gd, gtd = a.toarray(), g.toarray(), gt.toarray()
    aa, ga, gta = abs(ad), abs(gd), abs(gtd)
    na, ng, ngt = _max_row_terms(a), _max_row_terms(g), _max_row_terms(gt)
    carry, scale = chebyshev.cheb4_coefficients(beta, k)
    n = x_out.shape[0]
    nrm = lambda v: float(np.linalg.norm(v))  # noqa: E731
    n_gtg = np.linalg.norm(gtd @ gd, 2)
    n_gt = np.linalg.norm(gtd, 2)
    ma = gtd @ gd @ ad
    eye = np.eye(n)
    # the iterates x^_{-1}, x^_0, ..., x^_{k-1}
    iters = ([np.zeros(n)] + xs + [x_out]) if x0 is None else (xs + [x_out])
    assert len(iters) == k + 1 and len(rs) == k
    # local error norms of each step
    loc_u, loc_x = [], []
    d_prev = np.zeros(n)
    for i in range(k):
        xp, xn, r = iters[i], iters[i + 1], rs[i]
        if x0 is None and i == 0:
            f_r = 0.0   # the first residual is b itself
        else:
            f_r = nrm(_gamma(na, u) * (aa @ abs(xp)) + _gamma(1, u) * abs(r))
        f_t = nrm(_gamma(ng, u) * (ga @ abs(r)))
        f_z = nrm(_gamma(ngt, u) * (gta @ abs(ts[i])))
        c, s = (0.0 if i == 0 else carry[i]), scale[i]
        f_d = nrm(_gamma(4, u) * (abs(c) * d_prev + abs(s) * abs(zs[i])))
        loc_u.append(abs(s) * (n_gtg * f_r + n_gt * f_t + f_z) + f_d)
        loc_x.append(nrm(_gamma(1, u) * abs(xn)))
        # |delta^_i| from the two iterates it joins: x^_i = fl(x^_{i-1} + delta^_i)
        d_prev = abs(xn - xp) + 2.0 * _gamma(1, u) * abs(xn)
    # propagation: state (E_x, E_d); the product of the transitions after step i
    total = 0.0
    prod = np.eye(2 * n)
    for i in range(k - 1, -1, -1):
        top = prod[:n]   # [I 0] times the transitions after step i
        total += np.linalg.norm(top[:, :n] + top[:, n:], 2) * loc_u[i] + np.linalg.norm(top[:, :n], 2) * loc_x[i]
        c, s = (0.0 if i == 0 else carry[i]), scale[i]
        t = np.block([[eye - s * ma, c * eye], [-s * ma, c * eye]])
        prod = prod @ t
    return 1.01 * total


@functools.lru_cache(maxsize=None)
def _level(b, pw, shift, n=8):
    """One smoothed level (and its coarse level) of the PUM-shaped operator,
    with shift * max_i sum_j |a_ij| added to the diagonal when shift > 0 (a
    well-conditioned operator of the same structure, on which the bound is
    tight enough to tell a BF16 G from an FP32 one). Cached: the tests only
    read the hierarchy."""
    p = make_problem(n, 2, b, pw, seed=0)
    a = from_problem(p)
    if shift:
        sigma = shift * float(abs(a.scipy()).sum(axis=1).max())
        for k in range(a.nb):
            for e in range(a.rowptr[k], a.rowptr[k + 1]):
                if a.colidx[e] == k:
                    a.vals[e] = a.vals[e] + sigma * np.eye(b)
    sizes = grid_sizes(n, 2)
    starts = lanczos_starts(0, [s * s * b for s in sizes])
    levels = solver.build_levels(a, [prolongator(sizes[1], 2)], starts, "adaptive", 4)
    return p, levels, starts


@pytest.mark.parametrize("b,pw", [(3, 2), (10, 2)])
@pytest.mark.parametrize("store", ["f32", "bf16"])
@pytest.mark.parametrize("k,zero", [(1, True), (4, True), (4, False), (2, False)])
@pytest.mark.parametrize("shift", [0.0, 0.2])
def test_mixed_smoother_within_rounding_bound(b, pw, store, k, zero, shift):
    p, levels, starts = _level(b, pw, shift)
    ml = mixed.mixed_levels(levels, store, starts)
    lev, lev64 = ml[0], levels[0]
    n = p.ndof
    bv = rhs(0, n).astype(np.float32).astype(np.float64)
    x0 = None if zero else np.random.default_rng(1).standard_normal(n).astype(np.float32).astype(np.float64)
    # the oracle's mixed evaluation (FP32 operators, FP32 vectors)
    rec32 = _run(lev.a, lev.g, lev.gt, bv, x0, lev.beta, k, np.float32)
    # the exact smoother on the rounded operators, rounded independently and
    # evaluated in FP64
    def ref_ops(g_store):
        a64 = sp.bsr_matrix((_round_torch(lev64.a.vals, "f32"), lev64.a.colidx, lev64.a.rowptr), shape=(n, n))
        g64 = sp.bsr_matrix((_round_torch(lev64.g.vals, g_store), lev64.g.colidx, lev64.g.rowptr), shape=(n, n))
        return a64, g64, g64.T.tobsr(blocksize=(b, b))
    a64, g64, gt64 = ref_ops(store)
    rec64 = _run(a64, g64, gt64, bv, x0, lev.beta, k, np.float64)
    e32 = _bound(a64, g64, gt64, x0, lev.beta, k, rec32, U32)
    e64 = _bound(a64, g64, gt64, x0, lev.beta, k, rec64, U64)
    diff = float(np.linalg.norm(rec32[0] - rec64[0]))
    bound = e32 + e64
    assert diff <= bound, (diff, bound)
    # the bound is not vacuous: it stays well below the size of the result
    # (observed: 1e-3 to 6e-3 of it on the PUM operator, where the residual
    # cancels heavily, and 6e-5 to 1.4e-3 with the shift; the difference itself
    # is 3e-7 to 1e-6; a nonzero start adds |A||x0| to the first residual)
    size = float(np.linalg.norm(rec64[0]))
    assert bound < (2e-2 if shift == 0.0 else 5e-3) * size, (bound, size)
    # the computed result really carries FP32 rounding (not evaluated in FP64)
    assert diff > 0.0
    if store == "bf16" and shift > 0.0:
        # against the FP32-G exact smoother the BF16-G evaluation is outside
        # the bound: the BF16 rounding of G is part of what the oracle computes
        a6, g6, gt6 = ref_ops("f32")
        rec6 = _run(a6, g6, gt6, bv, x0, lev.beta, k, np.float64)
        wrong = float(np.linalg.norm(rec32[0] - rec6[0]))
        assert wrong > e32 + _bound(a6, g6, gt6, x0, lev.beta, k, rec6, U64), (wrong, e32)


def _smoother_propagator(ma, beta, k):
    """Exact map from the error of the start vector to the error of the
    result of Algorithm 3 (increment form, E_d starts at zero)."""
    n = ma.shape[0]
    carry, scale = chebyshev.cheb4_coefficients(beta, k)
    eye = np.eye(n)
    prod = np.eye(2 * n)
    for i in range(k - 1, -1, -1):
        c, s = (0.0 if i == 0 else carry[i]), scale[i]
        prod = prod @ np.block([[eye - s * ma, c * eye], [-s * ma, c * eye]])
    return prod[:n, :n]


@pytest.mark.parametrize("b", [3, 10])
@pytest.mark.parametrize("store", ["f32", "bf16"])
@pytest.mark.parametrize("shift", [0.0, 0.2])
@pytest.mark.parametrize("source", ["random", "coarse"])
@pytest.mark.parametrize("k", [1, 3])
def test_mixed_vcycle_within_rounding_bound(monkeypatch, b, store, shift, source, k):
    """V(k,k) of the mixed hierarchy (two levels; FP32 smoothing, residual,
    restriction and prolongation; FP64 Cholesky of the coarse Galerkin
    operator fed with FP32 data, its result rounded to FP32) against the
    exact cycle with the same stored operators. Local errors of each stage
    (the smoother bounds above; gamma_n |P^T||r^| and gamma_n |P||x^_c| for
    the transfers; Higham Thm. 10.4, |dA| <= gamma_{3n+1} |R^T||R| in FP64,
    for the Cholesky solve, plus one FP32 rounding of its result) are carried
    to the output by the exact maps of the stages after them. The "coarse"
    right-hand side is A P v_c, whose solution lies in the coarse space, so
    that the coarse correction carries a large part of the result (about a
    quarter at k = 1 on these grids: there a coarse correction off by 1%
    falls outside the bound)."""
    p, levels, starts = _level(b, 2, shift)
    ml = mixed.mixed_levels(levels, store, starts)
    lev, lev64 = ml[0], levels[0]
    assert lev.t is None and len(ml) == 2
    n = p.ndof
    # record what the cycle passes through the smoother and the transfers
    smooth_recs, restr, prol = [], [], []
    orig = chebyshev.cheb4

    def rec_cheb4(apply_a, apply_m, bb, x0, beta, kk, x_is_zero=False):
        xs, rs, ts, zs = [], [], [], []

        def aa(v):
            xs.append(np.asarray(v, dtype=np.float64).copy())
            return apply_a(v)

        def mm(v):
            rs.append(np.asarray(v, dtype=np.float64).copy())
            t = lev.g @ v
            ts.append(np.asarray(t, dtype=np.float64).copy())
            z = lev.gt @ t
            zs.append(np.asarray(z, dtype=np.float64).copy())
            return z

        x = orig(aa, mm, bb, x0, beta, kk, x_is_zero=x_is_zero)
        x0r = None if x_is_zero else np.asarray(x0, dtype=np.float64).copy()
        smooth_recs.append((x0r, (np.asarray(x, dtype=np.float64), xs, rs, ts, zs)))
        return x

    r_orig, p_orig = lev.restrict, lev.prolong

    def rec_restrict(r):
        out = r_orig(r)
        restr.append((np.asarray(r, dtype=np.float64).copy(), np.asarray(out, dtype=np.float64).copy()))
        return out

    def rec_prolong(xc):
        out = p_orig(xc)
        prol.append((np.asarray(xc, dtype=np.float64).copy(), np.asarray(out, dtype=np.float64).copy()))
        return out

    monkeypatch.setattr(mixed.chebyshev, "cheb4", rec_cheb4)
    monkeypatch.setattr(lev, "restrict", rec_restrict)
    monkeypatch.setattr(lev, "prolong", rec_prolong)
    if source == "random":
        bv = rhs(0, n).astype(np.float32)
    else:
        pfull = sp.kron(lev64.p_s, sp.identity(b), format="csr")
        bv = (lev64.a.scipy() @ (pfull @ rhs(1, pfull.shape[1]))).astype(np.float32)
    x_mixed = np.asarray(mixed.vcycle_mixed(ml, 0, bv, k), dtype=np.float64)
    monkeypatch.undo()
    assert len(smooth_recs) == 2 and len(restr) == 1 and len(prol) == 1

    # the stored operators, rounded independently, and the exact cycle on them
    def ops(g_store):
        a64 = sp.bsr_matrix((_round_torch(lev64.a.vals, "f32"), lev64.a.colidx, lev64.a.rowptr), shape=(n, n))
        g64 = sp.bsr_matrix((_round_torch(lev64.g.vals, g_store), lev64.g.colidx, lev64.g.rowptr), shape=(n, n))
        pb = sp.kron(lev64.p_s, sp.identity(b), format="csr")
        pb = sp.csr_matrix((_round_torch(pb.data, "f32"), pb.indices, pb.indptr), shape=pb.shape)
        return a64, g64, g64.T.tobsr(blocksize=(b, b)), pb

    ac = levels[1].a.dense()
    ac_inv = np.linalg.inv(ac)
    b64 = bv.astype(np.float64)

    def exact_cycle(a64, g64, gt64, pb):
        ad, gd = a64.toarray(), g64.toarray()
        ma = gd.T @ gd @ ad
        pd = pb.toarray()
        e_s = _smoother_propagator(ma, lev.beta, k)
        # the smoother from zero is (I - E_s) A^{-1} b; written without A^{-1}
        # through the recurrence itself, in FP64
        apply_a = lambda v: a64 @ v  # noqa: E731
        apply_m = lambda v: gt64 @ (g64 @ v)  # noqa: E731
        x1 = orig(apply_a, apply_m, b64, None, lev.beta, k, x_is_zero=True)
        x2 = x1 + pd @ np.linalg.solve(ac, pd.T @ (b64 - a64 @ x1))
        x3 = orig(apply_a, apply_m, b64, x2, lev.beta, k)
        return x3, ad, pd, e_s

    a64, g64, gt64, pb = ops(store)
    x_ref, ad, pd, e_post = exact_cycle(a64, g64, gt64, pb)

    u = U32
    nrm = lambda v: float(np.linalg.norm(v))  # noqa: E731
    n2 = lambda m: float(np.linalg.norm(m, 2))  # noqa: E731
    (x0_pre, rec_pre), (x0_post, rec_post) = smooth_recs
    assert x0_pre is None
    b_pre = _bound(a64, g64, gt64, None, lev.beta, k, rec_pre, u)
    b_post = _bound(a64, g64, gt64, x0_post, lev.beta, k, rec_post, u)
    x1 = rec_pre[0]
    r_in, _ = restr[0]
    xc, _ = prol[0]
    # stage errors
    na, npt, npr = _max_row_terms(a64), _max_row_terms(pb.T), _max_row_terms(pb)
    f_r = nrm(_gamma(na, u) * (abs(ad) @ abs(x1)) + _gamma(1, u) * abs(r_in))
    f_p = nrm(_gamma(npt, u) * (abs(pd).T @ abs(r_in)))
    nc = ac.shape[0]
    rfac = np.linalg.cholesky(ac).T
    f_c = n2(ac_inv) * nrm(_gamma(3 * nc + 1, U64) * (abs(rfac.T) @ (abs(rfac) @ abs(xc)))) + nrm(_gamma(1, u) * abs(xc))
    f_y = nrm(_gamma(npr, u) * (abs(pd) @ abs(xc)))
    x2 = x0_post
    f_add = nrm(_gamma(1, u) * abs(x2))
    coarse = pd @ ac_inv @ pd.T
    bound = (n2(e_post @ (np.eye(n) - coarse @ ad)) * b_pre + n2(e_post @ coarse) * f_r
             + n2(e_post @ pd @ ac_inv) * f_p + n2(e_post @ pd) * (f_c + f_y) + n2(e_post) * f_add + b_post)
    # the FP64 evaluation of the reference: far below the FP32 terms
    bound = 1.01 * bound + 1e-12 * nrm(x_ref)
    diff = nrm(x_mixed - x_ref)
    size = nrm(x_ref)
    assert diff <= bound, (diff, bound)
    assert 0.0 < diff and bound < (1e-1 if shift == 0.0 else 5e-3) * size, (diff, bound, size)
    if store == "bf16" and shift > 0.0:
        x_wrong = exact_cycle(*ops("f32"))[0]
        assert nrm(x_mixed - x_wrong) > bound, (nrm(x_mixed - x_wrong), bound)
