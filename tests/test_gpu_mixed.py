"""Mixed precision (A and G stored in FP32, G optionally BF16, FP32 vectors
and accumulation inside the V-cycle, FP64 outer PCG): per-application error
against the FP64 oracle and convergence of the outer PCG. The oracle's FP32
smoother and mixed cycle are pinned by rounding-error bounds
(test_oracle_mixed_bound.py). The bounds below follow from
the unit roundoffs (FP32 6e-8, BF16 3.9e-3) times the smoother's modest
amplification."""
import numpy as np
import pytest

from oracle import chebyshev, fsai, lanczos, multilevel, solver
from oracle.bsr import Bsr, from_problem
from oracle.mixed import round_bf16, round_f32
from problems import lanczos_starts, make_problem, rhs
from tests.helpers import dev, gpu_levels, hierarchy_inputs, host, rel_err, upload

pytestmark = pytest.mark.gpu

# b = 21 (triharmonic-like, 32x32) bounds for one application, against the
# FP64 oracle (FP32 storage; BF16 G) and against the oracle run on the rounded
# operators (what FP32 arithmetic adds). Observed on the MI355X: 3.3e-6,
# 3.7e-4 and 3.3e-6; the bounds leave a factor of about 6 to 13, as the b = 10
# ones do (observed 4.1e-7, 4.0e-4, 3.9e-7). The BF16 term is the BF16 unit
# roundoff (3.9e-3) scaled by how much of G's rounding survives the smoother.
TOL21_F32, TOL21_BF16, TOL21_R = 2e-5, 5e-3, 2e-5


@pytest.fixture(scope="module")
def chf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2509_06744_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("b,pw,store,tol_fp64,tol_rounded", [
    (10, 2, 1, 2e-5, 2e-5), (10, 2, 2, 5e-2, 2e-5), (21, 3, 1, TOL21_F32, TOL21_R), (21, 3, 2, TOL21_BF16, TOL21_R)])
def test_mixed_smoother_error(chf, b, pw, store, tol_fp64, tol_rounded):
    """One application (degree 4, x0 = 0) on a 32x32 grid: biharmonic-like
    b = 10 and triharmonic-like b = 21 (the mixed workload's block size)."""
    import torch
    p = make_problem(32, 2, b, pw, seed=0)
    a = from_problem(p)
    prow, pcol = fsai.pattern_lower(a)
    og = fsai.fsai(a, prow, pcol)
    asp, gsp = a.scipy(), og.scipy()
    gtsp = gsp.T.tocsr()
    beta, _ = lanczos.lmax(lambda v: gsp @ (asp @ (gtsp @ v)), lanczos_starts(0, [p.ndof])[0])
    b_ = rhs(0, p.ndof)
    want = chebyshev.cheb4(lambda v: asp @ v, lambda v: gtsp @ (gsp @ v), b_, None, beta, 4, x_is_zero=True)
    # the same algorithm on the rounded operators, evaluated in FP64
    ar = Bsr(a.rowptr, a.colidx, round_f32(a.vals), b).scipy()
    rg = round_bf16 if store == 2 else round_f32
    gr = Bsr(og.rowptr, og.colidx, rg(og.vals), b).scipy()
    grt = gr.T.tocsr()
    want_r = chebyshev.cheb4(lambda v: ar @ v, lambda v: grt @ (gr @ v), b_, None, beta, 4, x_is_zero=True)
    A = upload(p)
    G = chf.fsai_setup(A, chf.pattern_lower(A), g_store=store)
    x = torch.zeros(p.ndof, dtype=torch.float32, device="cuda")
    work = torch.zeros(3 * p.ndof, dtype=torch.float32, device="cuda")
    chf.cheb4_smooth(A, G, beta, 4, dev(b_, torch.float32), x, x_is_zero=True, work=work, dtype=store)
    e64 = rel_err(host(x), want)
    er = rel_err(host(x), want_r)
    print(f"b={b} store={store}: error vs FP64 oracle {e64:.3e}, vs rounded-operator oracle {er:.3e}")
    assert e64 < tol_fp64 and er < tol_rounded


@pytest.mark.parametrize("store", [1, 2])
def test_mixed_lanczos_on_rounded_operators(chf, store):
    p = make_problem(16, 2, 10, 2, seed=0)
    a = from_problem(p)
    prow, pcol = fsai.pattern_lower(a)
    og = fsai.fsai(a, prow, pcol)
    rg = round_bf16 if store == 2 else round_f32
    ar = Bsr(a.rowptr, a.colidx, round_f32(a.vals), 10).scipy()
    gr = Bsr(og.rowptr, og.colidx, rg(og.vals), 10).scipy()
    grt = gr.T.tocsr()
    v0 = lanczos_starts(0, [p.ndof])[0]
    want, wt = lanczos.lmax(lambda v: gr @ (ar @ (grt @ v)), v0)
    A = upload(p)
    G = chf.fsai_setup(A, chf.pattern_lower(A), g_store=store)
    beta, theta = chf.lmax_lanczos(A, G, dev(v0), dtype=store)
    assert abs(theta - wt) < 1e-8 * wt


@pytest.mark.parametrize("store", [1, 2])
def test_mixed_pcg_converges(chf, store):
    import torch
    p = make_problem(32, 2, 10, 2, seed=0)
    b_ = rhs(0, p.ndof)
    A64, L64, _, _ = gpu_levels(p, 3, 3, 0)
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    it64, _, _, _ = chf.pcg_solve(L64, dev(b_), x, rtol=1e-8, maxit=100)
    A, L, _, _ = gpu_levels(p, 3, 3, 0, dtype=store)
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    it, hist, tr, _ = chf.pcg_solve(L, dev(b_), x, rtol=1e-8, maxit=100, flexible=True)
    print(f"store={store}: PCG iterations FP64 {it64}, mixed {it}, true relres {tr:.2e}")
    assert hist[-1] <= 1e-8 and tr < 1e-7
    assert it <= it64 + (2 if store == 1 else 8)


@pytest.mark.parametrize("dt,name", [(0, "fp64"), (1, "mixed_f32"), (2, "mixed_bf16g"), (3, "fp64_bf16g")])
def test_triharmonic_pcg_matches_oracle_count(chf, dt, name):
    """b = 21 triharmonic-like (D = L^3) on 32x32 patches, 3 levels with the
    cubic patch transfer, adaptive t_max 8, V(4,4), PCG to a recursive 1e-10:
    within one iteration of the oracle's count for the same form
    (tests/golden/c2_n32_pcg_iterations.json, from the oracle alone)."""
    import json
    import os

    import torch
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_n32_pcg_iterations.json")) as f:
        gold = json.load(f)["dirichlet"]["pcg"][name]
    p = make_problem(32, 2, 21, 3, seed=0)
    b_ = rhs(0, p.ndof)
    A, L, _, _ = gpu_levels(p, 3, 4, 1, tmax=8, dtype=dt, order=4)
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda")
    it, hist, tr, _ = chf.pcg_solve(L, dev(b_), x, rtol=1e-10, maxit=300, flexible=dt in (1, 2))
    print(f"triharmonic {name}: {it} iterations (oracle {gold['iterations']}), true relres {tr:.2e} "
          f"(oracle {gold['true_relres']:.2e})")
    assert hist[-1] <= 1e-10
    assert abs(it - gold["iterations"]) <= 1


@pytest.mark.parametrize("store", [1, 2])
def test_b21_rounded_products(chf, store):
    """The b = 21 run layouts (FP32 A in runs of 4 and 1 columns, BF16 G in
    runs of 8, 8, 4, 1): A x and G^T G r against the oracle's products with the
    rounded operators, evaluated in FP64; FP32 accumulation bounds the error."""
    import torch
    p = make_problem(12, 2, 21, 3, seed=3)
    a = from_problem(p)
    prow, pcol = fsai.pattern_lower(a)
    og = fsai.fsai(a, prow, pcol)
    A = upload(p)
    G = chf.fsai_setup(A, chf.pattern_lower(A), g_store=store)
    x = np.random.default_rng(5).standard_normal(p.ndof)
    ar = Bsr(a.rowptr, a.colidx, round_f32(a.vals), 21).scipy()
    y = torch.zeros(p.ndof, dtype=torch.float32, device="cuda")
    chf.bsr_spmv(A, dev(x, torch.float32), y, dtype=1)
    assert rel_err(host(y), ar @ round_f32(x)) < 1e-5
    rg = round_bf16 if store == 2 else round_f32
    gr = Bsr(og.rowptr, og.colidx, rg(og.vals), 21).scipy()
    z = torch.zeros(p.ndof, dtype=torch.float32, device="cuda")
    w = torch.zeros(p.ndof, dtype=torch.float32, device="cuda")
    chf.fsai_apply(G, dev(x, torch.float32), z, w, dtype=store)
    assert rel_err(host(z), gr.T @ (gr @ round_f32(x))) < 1e-5


@pytest.mark.parametrize("n,b,pw,x_is_zero", [(24, 10, 2, True), (24, 10, 2, False), (16, 21, 3, True)])
def test_fp64_bf16g_smoother_matches_oracle(chf, n, b, pw, x_is_zero):
    """FP64 A, vectors and arithmetic with G read from its BF16 copy: the
    oracle runs the same FP64 algorithm on the BF16-rounded G, so the
    application matches it to the FP64 bar (1e-12); the Lanczos bound on the
    rounded factor matches too."""
    import torch
    p = make_problem(n, 2, b, pw, seed=0)
    a = from_problem(p)
    prow, pcol = fsai.pattern_lower(a)
    og = fsai.fsai(a, prow, pcol)
    asp = a.scipy()
    gr = Bsr(og.rowptr, og.colidx, round_bf16(og.vals), b).scipy()
    grt = gr.T.tocsr()
    v0 = lanczos_starts(0, [p.ndof])[0]
    beta, theta = lanczos.lmax(lambda v: gr @ (asp @ (grt @ v)), v0)
    b_ = rhs(0, p.ndof)
    x0 = np.random.default_rng(2).standard_normal(p.ndof)
    want = chebyshev.cheb4(lambda v: asp @ v, lambda v: grt @ (gr @ v), b_, None if x_is_zero else x0, beta, 4,
                           x_is_zero=x_is_zero)
    A = upload(p)
    G = chf.fsai_setup(A, chf.pattern_lower(A), g_store=chf.BF16)
    gb, gt = chf.lmax_lanczos(A, G, dev(v0), dtype=chf.F64_BF16G)
    assert abs(gt - theta) < 1e-9 * theta
    x = torch.zeros(p.ndof, dtype=torch.float64, device="cuda") if x_is_zero else dev(x0)
    work = torch.zeros(3 * p.ndof, dtype=torch.float64, device="cuda")
    chf.cheb4_smooth(A, G, beta, 4, dev(b_), x, x_is_zero=x_is_zero, work=work, dtype=chf.F64_BF16G)
    assert rel_err(host(x), want) < 1e-12
