"""Benchmark: fourth-kind Chebyshev / block-FSAI smoother throughput and
V-cycle-preconditioned PCG time to 1e-8, FP64 vs mixed, on one MI355X.

Workload (default): biharmonic-like 2D, 512 x 512 patches, b = 10
(2,621,440 dofs), A = R^T (L^2 (x) I_b) R, adaptive block-FSAI with
t_max = 8 (Algorithm 1, tau = 1, P0 = diagonal), Chebyshev degree 4,
6-level Galerkin V(4,4), RHS N(0,1) with seed 0. Inputs are seeded synthetic
data generated on the host and resident in HBM before any timed region.

Timed steps: one step is one smoother application (Algorithm 3, degree 4,
x != 0) on level 0: the hot loop of every V-cycle. `value` = N * k / t_app in
GDOF/s. The PCG solves (FP64 and mixed) and the set-up phases are timed in
the same run and reported beside it.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_NOTE = os.path.join(ROOT, "profiles", "k_sell_spmv_residual_512x512_b10_traffic.md")
SPMV_SOURCE = os.path.join(ROOT, "paper_2509_06744_amd", "csrc", "bsr.hip")


KERNEL_STATS = os.path.join(ROOT, "profiles", "bench_512x512_b10_kernel_stats.md")
GOLDEN_C1 = os.path.join(ROOT, "tests", "golden", "c1_pcg_iterations.json")


def rocprof_residual_avg_ms():
    """rocprofv3's average duration of the timed residual SpMV dispatches from
    the committed kernel-statistics summary, or None when the SpMV source
    changed since it was taken."""
    import hashlib
    try:
        note = open(KERNEL_STATS).read()
        sha = hashlib.sha256(open(SPMV_SOURCE, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    if f"sha256 prefix {sha}" not in note:
        return None
    for line in note.splitlines():
        if line.startswith("rocprof_timed_avg_us:"):
            return float(line.split(":", 1)[1]) / 1e3
    return None


def measured_traffic():
    """HBM bytes per launch of the residual SpMV from the committed counter
    summary, or None when the kernel source changed since it was measured."""
    import hashlib
    try:
        note = open(TRAFFIC_NOTE).read()
        sha = hashlib.sha256(open(SPMV_SOURCE, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    fields = dict(line.split(": ", 1) for line in note.splitlines() if line.startswith(("traffic_", "kernel_")))
    if fields.get("kernel_source_sha256_prefix", "").strip() != sha:
        return None
    return float(fields["traffic_bytes_per_launch"])


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=512, help="patches per side")
    ap.add_argument("--levels", type=int, default=6)
    ap.add_argument("--tmax", type=int, default=8)
    ap.add_argument("--degree", type=int, default=4)
    ap.add_argument("--no-pcg", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-comparators", action="store_true")
    ap.add_argument("--no-nested", action="store_true")
    ap.add_argument("--no-setup3d", action="store_true")
    ap.add_argument("--no-c2", action="store_true", help="skip the mixed-precision triharmonic (b = 21) leg")
    ap.add_argument("--only-c2", action="store_true", help="run only the triharmonic leg")
    ap.add_argument("--setup3d-grid", type=int, default=64, help="3D patch grid of the batched set-up leg")
    ap.add_argument("--setup3d-tmax", type=int, default=23)
    ap.add_argument("--only-setup3d", action="store_true",
                    help="run only the batched 3D set-up leg (for hardware-counter passes)")
    ap.add_argument("--train-seeds", type=int, default=32, help="training seeds 1..S")
    ap.add_argument("--test-seeds", type=int, default=8, help="test seeds 100..100+T-1 (up to 8)")
    ap.add_argument("--cpu-grid", type=int, default=32, help="patches per side of the oracle's timing sample")
    ap.add_argument("--only-spmv", action="store_true",
                    help="build A only and run the level-0 residual SpMV (for hardware-counter passes)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run 3 plain device copies of 1 GiB (reference for HBM counters)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(n, b, tmax, degree, target_s=10.0, levels=3):
    """The oracle (plain FP64 NumPy/SciPy) on a bounded sample of the same
    workload: a smaller patch grid of the same generator, block size, adaptive
    pattern, degree and smoother. The headline value times the smoother
    applications; beside it, each labelled, the oracle's Algorithm 1 and block
    FSAI set-up on that grid, the rest of a `levels`-level hierarchy
    (Galerkin products, Lanczos bounds, coarse factor) and PCG to 1e-8 with
    V(degree, degree)."""
    from oracle import adaptive, chebyshev, fsai, lanczos, multilevel
    from oracle.bsr import from_problem
    from problems import grid_sizes, lanczos_starts, level_basis, make_problem, prolongator, rhs
    p = make_problem(n, 2, b, 2, seed=0)
    a = from_problem(p)
    sizes = grid_sizes(n, levels)
    starts = lanczos_starts(0, [s_ * s_ * b for s_ in sizes])
    t0 = time.perf_counter()
    prow, pcol = adaptive.adaptive_pattern(a, tmax)
    pattern_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    g = fsai.fsai(a, prow, pcol)
    fsai_s = time.perf_counter() - t0
    asp, gsp = a.scipy(), g.scipy()
    gtsp = gsp.T.tocsr()
    beta, _ = lanczos.lmax(lambda v: gsp @ (asp @ (gtsp @ v)), starts[0])
    bvec = rhs(0, p.ndof)
    x = np.zeros(p.ndof)
    reps = 0
    t0 = time.perf_counter()
    while True:
        x = chebyshev.cheb4(lambda v: asp @ v, lambda v: gtsp @ (gsp @ v), bvec, x, beta, degree)
        reps += 1
        el = time.perf_counter() - t0
        if el >= target_s or reps >= 100000:
            break
    t_app = el / reps
    # the rest of the hierarchy, then PCG (level 0 reuses the pattern and factor above)
    t0 = time.perf_counter()
    pro = [prolongator(sizes[l + 1], 2) for l in range(levels - 1)]
    bases = level_basis(p, levels)
    hier, al = [], a
    for l in range(levels):
        lev = multilevel.Level(a=al)
        if l == levels - 1:
            lev.finish()
            lev.chol = multilevel.coarse_factor(al)
            hier.append(lev)
            break
        if l == 0:
            lev.g = g
        else:
            pr, pc = adaptive.adaptive_pattern(al, tmax)
            lev.g = fsai.fsai(al, pr, pc)
        lev.p_s, lev.basis = pro[l], bases[l]
        lev.finish()
        lev.beta, _ = lanczos.lmax(lev.apply_b, np.asarray(starts[l]), 100, 1.01)
        hier.append(lev)
        al = multilevel.galerkin(al, pro[l], bases[l])
    hier_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, pcg_it, _, pcg_tr = multilevel.pcg(hier[0].apply_a, lambda r: multilevel.vcycle(hier, 0, r, degree), bvec,
                                          1e-8, 300)
    pcg_s = time.perf_counter() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except Exception:
        cores = os.cpu_count()
    threads = os.environ.get("OMP_NUM_THREADS", "unset")
    return {
        "value": p.ndof * degree / t_app / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
        "sample": (f"{reps} oracle smoother applications (Algorithm 3, degree {degree}, SciPy BSR products, "
                   f"single-threaded) on a {n}x{n}-patch grid of the same generator (b={b}, {p.ndof} dofs, "
                   f"adaptive t_max={tmax}); {el:.1f} s timed; "
                   f"host affinity {cores} cores, OMP_NUM_THREADS={threads}"),
        "oracle_setup_and_solve": {
            "grid": f"{n}x{n} patches, b={b}, {p.ndof} dofs, {levels} levels, V({degree},{degree})",
            "adaptive_pattern_s": round(pattern_s, 2),
            "fsai_setup_s": round(fsai_s, 2),
            "fsai_setup_rows_per_s": round(p.nb / fsai_s, 1),
            "rest_of_hierarchy_s": round(hier_s, 2),
            "pcg_iterations": int(pcg_it),
            "pcg_s": round(pcg_s, 2),
            "pcg_true_relres": float(pcg_tr),
            "note": "plain Python/NumPy/SciPy row loops, one core; not the GPU path's algorithms or layout",
        },
    }


def cpu_setup3d_sample(g, b, tmax, target_s=10.0, max_rows=4096):
    """The oracle's Algorithm 1 and block-FSAI set-up on a sample of rows of
    the 3D set-up workload (g^3 patches, t_max from P0 = diagonal), beside
    the GPU's whole-matrix times: rows spread evenly over the middle third of
    the grid (interior rows, the 262,064-of-262,144 majority at 64^3), taken
    in a fixed stratified order until about target_s seconds have passed; a
    per-row rate, labelled as a sample."""
    from oracle import adaptive, fsai
    from oracle.bsr import from_problem
    from problems import make_problem
    t0 = time.perf_counter()
    a = from_problem(make_problem(g, 3, b, 2, seed=0))
    gen_s = time.perf_counter() - t0
    lo, span = a.nb // 3, a.nb // 3
    # strata: max_rows evenly spaced rows, visited in bit-reversed order so
    # that any prefix of the visit covers the middle third evenly
    nbits = max(1, (max_rows - 1).bit_length())
    order = [int(format(i, f"0{nbits}b")[::-1], 2) for i in range(1 << nbits)]
    order = [o for o in order if o < max_rows]
    pat_s = fsai_s = 0.0
    done, sizes = [], []
    for o in order:
        k = int(lo + o * span // max_rows)
        t0 = time.perf_counter()
        prow, pcol = adaptive.adaptive_pattern(a, tmax, rows=[k])
        pat_s += time.perf_counter() - t0
        t0 = time.perf_counter()
        fsai.fsai_row(a, k, pcol[prow[0]:prow[1]])
        fsai_s += time.perf_counter() - t0
        done.append(k)
        sizes.append(int(prow[1] - prow[0]))
        if pat_s + fsai_s >= target_s:
            break
    return {
        "sample": (f"sampled: {len(done)} interior rows of the {g}^3-patch workload (b={b}, {a.nb} block rows), "
                   f"evenly spread over the middle third, Algorithm 1 with t_max={tmax} from P0 = diagonal, "
                   "then each row's block-FSAI solve; plain Python/NumPy row loops, BLAS threads "
                   f"OMP_NUM_THREADS={os.environ.get('OMP_NUM_THREADS', 'unset')}"),
        "rows": len(done),
        "pattern_blocks_per_row_mean": round(float(np.mean(sizes)), 2),
        "adaptive_pattern_s_per_row": round(pat_s / len(done), 4),
        "fsai_setup_s_per_row": round(fsai_s / len(done), 5),
        "adaptive_pattern_rows_per_s": round(len(done) / pat_s, 2),
        "fsai_setup_rows_per_s": round(len(done) / fsai_s, 1),
        "generator_s": round(gen_s, 1),
    }


def setup3d_leg(args, chf, torch):
    """Batched block-FSAI set-up of the 3D biharmonic-like workload: Algorithm 1
    with t_max = 23 from P0 = diagonal gives local systems of 1..24 blocks
    (10..240 wide); all of them are factored in one persistent launch. FLOPs
    counted as sum_k (n_k^3 / 3 + n_k^2 b) (Cholesky plus the last-b-rows
    solve), against the FP64 MFMA peak."""
    from problems import make_problem
    g, b = args.setup3d_grid, 10
    q = make_problem(g, 3, b, 2, seed=0)
    Aq = chf.bsr_create(q.nb, q.b, q.rowptr, q.colidx, q.vals)
    torch.cuda.synchronize()
    t = time.perf_counter()
    P = chf.pattern_adaptive(Aq, args.setup3d_tmax)
    t_pat = time.perf_counter() - t
    rp, _ = chf.pattern_export(P)
    sizes = np.diff(rp) * b
    flops = float(np.sum(sizes.astype(np.float64) ** 3 / 3.0 + sizes.astype(np.float64) ** 2 * b))
    t = time.perf_counter()
    G = chf.fsai_setup(Aq, P)              # first call includes the autotuning of the solver configuration
    t_first = time.perf_counter() - t
    del G
    reps = 3
    t = time.perf_counter()
    for _ in range(reps):
        G = chf.fsai_setup(Aq, P)
        del G
    t_setup = (time.perf_counter() - t) / reps
    rec = {"grid": f"{g}^3", "block": b, "tmax": args.setup3d_tmax, "systems": int(q.nb),
           "local_size_hist": {str(int(s_)): int(c) for s_, c in zip(*np.unique(sizes, return_counts=True))},
           "adaptive_pattern_ms": round(1e3 * t_pat, 1), "fsai_setup_first_call_ms": round(1e3 * t_first, 1),
           "fsai_setup_ms": round(1e3 * t_setup, 2), "flops": flops,
           "achieved_TFLOPs": round(flops / t_setup / 1e12, 3), "peak_TFLOPs": 78.6,
           "frac": round(flops / t_setup / 1e12 / 78.6, 4),
           "note": "fsai_setup_ms is the whole call: local factorisations, G^T transpose map, SpMV layouts"}
    log(f"3D batched set-up: {rec}")
    return rec


def first_below(hist, tol):
    """First iteration whose recursive relative residual is <= tol, or None."""
    idx = np.nonzero(np.asarray(hist) <= tol)[0]
    return int(idx[0]) if idx.size else None


def c2_leg(args, chf, torch, dev):
    """Mixed-precision triharmonic workload: D = L^3 (25-point block stencil),
    256 x 256 patches, b = 21 (1,376,256 dofs), five Galerkin levels with the
    cubic patch transfer, adaptive block-FSAI t_max = 8, V(4,4) fourth-kind
    Chebyshev smoothing, outer FP64 PCG to a recursive relative residual of
    1e-10. Forms: A and G in FP32, A in FP32 with G in BF16 (flexible PCG), and
    the plain FP64 form for reference. For each: set-up and PCG time,
    iterations, the recursive and the true residual, one level-0 smoother
    application (median of 20 calls) against its algorithmic bytes, and that
    application's error against the FP64 form's on the same inputs."""
    from problems import CONFIGS, grid_sizes, lanczos_starts, level_basis, make_problem, prolongator, rhs
    cfg = CONFIGS["c2"]
    n, b, L, k = cfg.n, cfg.b, cfg.levels, cfg.degree
    p = make_problem(n, 2, b, cfg.power, seed=cfg.seed)
    sizes = grid_sizes(n, L)
    pro = [prolongator(sizes[l + 1], 2, cfg.transfer_order) for l in range(L - 1)]
    starts = lanczos_starts(cfg.seed, [s_ * s_ * b for s_ in sizes])
    bases = level_basis(p, L)
    bd = torch.from_numpy(rhs(cfg.seed, p.ndof)).to(dev)
    A = chf.bsr_create(p.nb, p.b, p.rowptr, p.colidx, p.vals)
    nnzb, N = p.nnzb, p.ndof
    v0 = [torch.from_numpy(s_).to(dev) for s_ in starts[:-1]]
    del p
    stream = torch.cuda.current_stream()
    out = {"workload": (f"triharmonic-like 2D PUM-shaped A=R^T(L^3 (x) I_b)R, {n}x{n} patches, b={b}, {N} dofs, "
                        f"{L}-level Galerkin V({k},{k}), cubic patch transfer, finest transfer "
                        f"P = R^-1 (P_s (x) I_b), adaptive t_max={cfg.tmax}, PCG rtol {cfg.rtol:g}"), "nnzb_A": nnzb}
    x64 = None
    for name, dt in [("fp64", chf.F64), ("mixed_f32", chf.F32), ("mixed_bf16g", chf.BF16),
                     ("fp64_bf16g", chf.F64_BF16G)]:
        rec = {}
        H = chf.levels_create(A)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for ps, basis in zip(pro, bases):
            chf.levels_add_coarse(H, ps.shape[1], ps.indptr, ps.indices, ps.data, basis)
        torch.cuda.synchronize()
        rec["galerkin_ms"] = round(1e3 * (time.perf_counter() - t), 1)
        t = time.perf_counter()
        chf.levels_setup(H, degree=k, pattern=1, tmax=cfg.tmax, dtype=dt, v0=v0)
        torch.cuda.synchronize()
        rec["levels_setup_ms"] = round(1e3 * (time.perf_counter() - t), 1)
        rec["blocks_per_row_A"] = []
        for l in range(L):
            Al, _, _ = chf.levels_get(H, l)
            nb_l, _, nz_l = Al.info()
            rec["blocks_per_row_A"].append(round(nz_l / nb_l, 1))
        flex = dt in (chf.F32, chf.BF16)
        # the FP32-A cycle stalls near a recursive 2e-9 on this operator: those
        # forms are run to 1e-8 (the biharmonic workload's target)
        rtol = 1e-8 if flex else cfg.rtol
        rec["rtol"] = rtol
        xs = torch.zeros(N, dtype=torch.float64, device=dev)
        chf.pcg_solve(H, bd, xs, rtol=rtol, maxit=400, flexible=flex, raise_on_noconv=False)   # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        it, hist, tr, rc = chf.pcg_solve(H, bd, xs, rtol=rtol, maxit=400, flexible=flex, raise_on_noconv=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        rec.update({"iterations": it, "time_ms": round(1e3 * el, 2), "ms_per_iteration": round(1e3 * el / max(it, 1), 3),
                    "final_relres": float(hist[-1]), "true_relres": tr, "converged": rc == 0, "flexible_cg": flex,
                    "iterations_to": {f"{t:g}": first_below(hist, t) for t in (1e-6, 1e-8, 1e-10)}})
        # one level-0 smoother application with this form's operators, x0 = 0
        A0, G0, P0 = chf.levels_get(H, 0)
        beta0 = chf.levels_get_beta(H, 0)
        _, pcol = chf.pattern_export(P0)
        nnzg = len(pcol)
        vt = torch.float64 if dt in (chf.F64, chf.F64_BF16G) else torch.float32
        bb_ = bd.to(vt)
        x = torch.zeros(N, dtype=vt, device=dev)
        work = torch.zeros(3 * N, dtype=vt, device=dev)
        for _ in range(3):
            chf.cheb4_smooth(A0, G0, beta0, k, bb_, x, x_is_zero=False, work=work, dtype=dt)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(20)]
        for a_, b_ in evs:
            a_.record(stream)
            chf.cheb4_smooth(A0, G0, beta0, k, bb_, x, x_is_zero=False, work=work, dtype=dt)
            b_.record(stream)
        torch.cuda.synchronize()
        ms = float(np.median([a_.elapsed_time(b_) for a_, b_ in evs]))
        sa, sv = (8, 8) if dt in (chf.F64, chf.F64_BF16G) else (4, 4)
        sg = 8 if dt == chf.F64 else (4 if dt == chf.F32 else 2)
        b_app = k * (nnzb * (b * b * sa + 4) + 2 * nnzg * (b * b * sg + 4) + 10 * N * sv)
        rec["smoother"] = {"median_ms_per_application_20_calls": round(ms, 4), "algorithmic_bytes_per_application": b_app,
                           "achieved_GBs": round(b_app / (ms * 1e-3) / 1e9, 1),
                           "hbm_frac": round(b_app / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                           "gdofs": round(N * k / (ms * 1e-3) / 1e9, 4), "nnzb_G": nnzg}
        # error of one application from x0 = 0 against the FP64 form's
        x.zero_()
        chf.cheb4_smooth(A0, G0, beta0, k, bb_, x, x_is_zero=True, work=work, dtype=dt)
        xd = x.double()
        if x64 is None:
            x64 = xd.clone()
        else:
            rec["smoother"]["rel_error_vs_fp64_application"] = float((xd - x64).abs().max() / x64.abs().max())
        out[name] = rec
        log(f"c2 {name}: {rec}")
        H.destroy()
        del work, x
    out["fp64_bf16g_over_fp64_time"] = round(out["fp64_bf16g"]["time_ms"] / out["fp64"]["time_ms"], 4)
    return out


def comparators_leg(args, chf, torch, dev, H, A, bd, N, k):
    """The smoothers and cycles that Sec. 3.1 and Sec. 5 compare, on the same
    FP64 hierarchy (same patterns, factors and bounds beta_l): fourth-kind
    Chebyshev, first-kind Chebyshev on [0.3 beta, beta], Richardson
    (omega = 1, S = (I - MA)^k), each in V(k,k), and fourth-kind Chebyshev in
    V(2k,0). For each: the energy-norm convergence factor of the cycle from a
    U(-1,1) error, and a Krylov solve to 1e-8: CG for the symmetric cycles,
    flexible CG and BiCGStab (two cycles per iteration) for V(2k,0), and
    BiCGStab with V(k,k) for reference."""
    from problems import uniform_start
    e0 = torch.from_numpy(uniform_start(0, N)).to(dev)
    runs = [("cheb4_Vkk", chf.SMOOTH_CHEB4, 0.0, chf.CYCLE_VKK),
            ("cheb1_rho0.3_Vkk", chf.SMOOTH_CHEB1, 0.3, chf.CYCLE_VKK),
            ("richardson_omega1_Vkk", chf.SMOOTH_RICHARDSON, 1.0, chf.CYCLE_VKK),
            ("cheb4_V2k0", chf.SMOOTH_CHEB4, 0.0, chf.CYCLE_V2K0),
            ("cheb4_V2k0_bicgstab", chf.SMOOTH_CHEB4, 0.0, chf.CYCLE_V2K0),
            ("cheb4_Vkk_bicgstab", chf.SMOOTH_CHEB4, 0.0, chf.CYCLE_VKK)]
    out = {}
    for name, sm, par, cyc in runs:
        chf.levels_set_cycle(H, sm, par, cyc)
        rec = {}
        bicg = name.endswith("_bicgstab")
        if not bicg:
            rho, ncyc = chf.levels_energy_factor(H, e0, maxit=30)
            rec["rho_A"], rec["cycles"] = round(rho, 5), ncyc
        flex = cyc == chf.CYCLE_V2K0
        xs = torch.zeros(N, dtype=torch.float64, device=dev)
        try:
            torch.cuda.synchronize()
            t = time.perf_counter()
            if bicg:
                it, hist, tr, rc = chf.bicgstab_solve(H, bd, xs, rtol=1e-8, maxit=200, raise_on_noconv=False)
            else:
                it, hist, tr, rc = chf.pcg_solve(H, bd, xs, rtol=1e-8, maxit=200, flexible=flex,
                                                 raise_on_noconv=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            rec.update({"solver": "bicgstab" if bicg else ("flexible_cg" if flex else "cg"),
                        "iterations": it, "time_ms": round(1e3 * el, 2),
                        "ms_per_iteration": round(1e3 * el / max(it, 1), 3), "converged": rc == 0,
                        "true_relres": tr, "preconditioner_applications": (2 * it if bicg else it)})
        except chf.ChfError as e:
            rec["pcg_error"] = str(e)
        out[name] = rec
        log(f"comparator {name}: {rec}")
    chf.levels_set_cycle(H, chf.SMOOTH_CHEB4, 0.0, chf.CYCLE_VKK)
    return out


def nested_leg(args, chf, torch, dev, A, bd, N, k, pro, bases, v0, H_plain, plain_setup_ms):
    """Nested block-FSAI (Sec. 2.2, one nesting level, Algorithm 1 with the same
    t_max on both levels) against plain FSAI with t_max = 8 on the same 512^2
    hierarchy: set-up time, energy-norm cycle factor, PCG to 1e-8 and the time
    of one level-0 smoother application (five kernels per step instead of
    three). Sec. 5 observes that nested t_max = c behaves like plain 2c."""
    from problems import uniform_start
    e0 = torch.from_numpy(uniform_start(0, N)).to(dev)
    out = {}

    def measure(H, name, setup_ms):
        rec = {"levels_setup_ms": round(setup_ms, 1)}
        rho, ncyc = chf.levels_energy_factor(H, e0, maxit=30)
        rec["rho_A"], rec["cycles"] = round(rho, 5), ncyc
        xs = torch.zeros(N, dtype=torch.float64, device=dev)
        chf.pcg_solve(H, bd, xs, rtol=1e-8, maxit=200, raise_on_noconv=False)
        torch.cuda.synchronize()
        t = time.perf_counter()
        it, hist, tr, rc = chf.pcg_solve(H, bd, xs, rtol=1e-8, maxit=200, raise_on_noconv=False)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        rec.update({"pcg_iterations": it, "pcg_time_ms": round(1e3 * el, 2), "converged": rc == 0,
                    "true_relres": tr})
        _, G0, _ = chf.levels_get(H, 0)
        beta0 = chf.levels_get_beta(H, 0)
        x = torch.zeros(N, dtype=torch.float64, device=dev)
        work = torch.zeros(3 * N, dtype=torch.float64, device=dev)
        for _ in range(2):
            chf.cheb4_smooth(A, G0, beta0, k, bd, x, x_is_zero=False, work=work)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(10):
            chf.cheb4_smooth(A, G0, beta0, k, bd, x, x_is_zero=False, work=work)
        ev1.record()
        torch.cuda.synchronize()
        rec["smoother_ms_per_application"] = round(ev0.elapsed_time(ev1) / 10, 4)
        out[name] = rec
        log(f"nested leg {name}: {rec}")

    measure(H_plain, f"plain_tmax{args.tmax}", plain_setup_ms)
    for tm in (4, 8):
        H = chf.levels_create(A)
        for ps, basis in zip(pro, bases):
            chf.levels_add_coarse(H, ps.shape[1], ps.indptr, ps.indices, ps.data, basis)
        chf.levels_set_nesting(H, 1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        chf.levels_setup(H, degree=k, pattern=1, tmax=tm, v0=v0)
        torch.cuda.synchronize()
        measure(H, f"nested_tmax{tm}", 1e3 * (time.perf_counter() - t))
        H.destroy()
    return out


def learned_leg(args, chf, torch, dev, n, b, L, k, pro, bases_unused):
    """Train the pattern proposer on Algorithm 1's patterns (seeds 1..S of the
    2D 64x64 and 3D 12^3 generators, b = 10, t_max = 8), then compare three
    level-0 patterns on the benchmark grid for seeds 100..107: Algorithm 1,
    the network's proposal, and the interior template (the offsets of
    Algorithm 1's pattern at the centre row of a 64x64 training grid, applied
    at every row). For each: the time to form the pattern, the share of rows
    identical to Algorithm 1's, and the V(k,k) energy-norm convergence factor
    with that pattern on level 0 (coarser levels use Algorithm 1 in every
    case)."""
    from paper_2509_06744_amd import learned
    from problems import lanczos_starts, level_basis, make_problem, mlp_init, permutation, uniform_start
    t0 = time.perf_counter()
    items, keep = [], []
    tmpl = None
    for seed in range(1, args.train_seeds + 1):
        for nn, dim in [(64, 2), (12, 3)]:
            q = make_problem(nn, dim, b, 2, seed=seed)
            Aq = chf.bsr_create(q.nb, q.b, q.rowptr, q.colidx, q.vals)
            Pq = chf.pattern_adaptive(Aq, args.tmax)
            items.append((Aq, nn, nn, Pq))
            keep.append((Aq, Pq))
            if tmpl is None and dim == 2:
                rp_, cp_ = chf.pattern_export(Pq)
                tmpl = learned.template_offsets(rp_, cp_, nn, nn, (nn // 2) * nn + nn // 2)
    X, Y = learned.dataset(items)
    t_data = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    perm = torch.from_numpy(permutation(0, Y.shape[0])).to(dev)
    net, hist = learned.train(X, Y, mlp_init(0), perm, epochs=4, batch=8192, lr=2e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del items, keep, X, Y
    tests = []
    for seed in range(100, 100 + min(8, args.test_seeds)):
        q = make_problem(n, 2, b, 2, seed=seed)
        Aq = chf.bsr_create(q.nb, q.b, q.rowptr, q.colidx, q.vals)
        starts = lanczos_starts(seed, [s * s * b for s in [n >> l for l in range(L)]])
        v0 = [torch.from_numpy(s_).to(dev) for s_ in starts[:-1]]
        e0 = torch.from_numpy(uniform_start(seed, q.ndof)).to(dev)
        qb = level_basis(q, L)
        rec = {"seed": seed}
        pats = {}
        for name, make in [("adaptive", lambda: chf.pattern_adaptive(Aq, args.tmax)),
                           ("learned", lambda: chf.mlp_propose(Aq, net, n, n, args.tmax)),
                           ("template", lambda: chf.pattern_template(n, n, 1, tmpl))]:
            best = None
            for _ in range(3):
                torch.cuda.synchronize()
                t = time.perf_counter()
                P = make()
                torch.cuda.synchronize()
                el = time.perf_counter() - t
                best = el if best is None else min(best, el)
            pats[name] = P
            rec[f"pattern_ms_{name}"] = round(1e3 * best, 2)
        ra, ca = chf.pattern_export(pats["adaptive"])
        for name in ("learned", "template"):
            rl, cl = chf.pattern_export(pats[name])
            same = sum(1 for kk in range(q.nb) if np.array_equal(ca[ra[kk]:ra[kk + 1]], cl[rl[kk]:rl[kk + 1]]))
            rec[f"rows_identical_{name}"] = round(same / q.nb, 4)
        for name, P in pats.items():
            H = chf.levels_create(Aq)
            for ps, basis in zip(pro, qb):
                chf.levels_add_coarse(H, ps.shape[1], ps.indptr, ps.indices, ps.data, basis)
            chf.levels_set_pattern(H, 0, P)
            t = time.perf_counter()
            chf.levels_setup(H, degree=k, pattern=1, tmax=args.tmax, v0=v0)
            torch.cuda.synchronize()
            rec[f"levels_setup_ms_{name}"] = round(1e3 * (time.perf_counter() - t), 1)
            rho, cyc = chf.levels_energy_factor(H, e0)
            rec[f"rho_A_{name}"] = round(rho, 5)
            rec[f"cycles_{name}"] = cyc
            H.destroy()
        tests.append(rec)
        log(f"learned vs adaptive vs template: {rec}")
        del q
    summ = {}
    for name in ("adaptive", "learned", "template"):
        summ[f"pattern_ms_{name}_mean"] = round(float(np.mean([t[f"pattern_ms_{name}"] for t in tests])), 2)
        summ[f"rho_A_{name}_mean"] = round(float(np.mean([t[f"rho_A_{name}"] for t in tests])), 5)
    for name in ("learned", "template"):
        summ[f"rows_identical_{name}_mean"] = round(float(np.mean([t[f"rows_identical_{name}"] for t in tests])), 4)
    return {"train": {"seeds": f"1..{args.train_seeds}", "grids": "64x64 2D and 12^3 3D, b=10, t_max=8",
                      "samples": int(len(perm)), "epochs": 4, "loss": [round(float(v), 5) for v in hist],
                      "data_s": round(t_data, 2), "train_s": round(t_train, 2)},
            "template_offsets": [list(map(int, o)) for o in tmpl],
            "test": tests, "summary": summ}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the path has no multi-GPU implementation "
              "(its sharding is described, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2509_06744_amd as chf
    from problems import grid_sizes, lanczos_starts, level_basis, make_problem, prolongator, rhs

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.only_setup3d:
        print(json.dumps({"setup3d": setup3d_leg(args, chf, torch)}), flush=True)
        return
    if args.only_c2:
        print(json.dumps({"c2": c2_leg(args, chf, torch, dev)}), flush=True)
        return
    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n, b, L, k = args.n, 10, args.levels, args.degree
    log(f"generating {n}x{n} b={b} problem")
    t0 = time.perf_counter()
    p = make_problem(n, 2, b, 2, seed=0)
    sizes = grid_sizes(n, L)
    pro = [prolongator(sizes[l + 1], 2) for l in range(L - 1)]
    starts = lanczos_starts(0, [s * s * b for s in sizes])
    bvec = rhs(0, p.ndof)
    bases = level_basis(p, L)
    log(f"generated in {time.perf_counter() - t0:.1f} s; uploading")
    torch.cuda.synchronize()   # device start-up is not part of the upload
    t_up = time.perf_counter()
    A = chf.bsr_create(p.nb, p.b, p.rowptr, p.colidx, p.vals)
    torch.cuda.synchronize()
    bsr_create_ms = 1e3 * (time.perf_counter() - t_up)   # host checks, PCIe upload of A, SpMV layout
    nnzb = p.nnzb
    v0 = [torch.from_numpy(s).to(dev) for s in starts[:-1]]
    bd = torch.from_numpy(bvec).to(dev)
    del p
    if args.only_spmv:
        N = A.info()[0] * b
        xs = torch.ones(N, dtype=torch.float64, device=dev)
        r = torch.empty_like(xs)
        for _ in range(args.steps):
            chf.bsr_spmv(A, xs, r, bvec=bd)
        torch.cuda.synchronize()
        print(json.dumps({"only_spmv": True, "launches": args.steps,
                          "algorithmic_bytes_per_launch": nnzb * (b * b * 8 + 4) + 3 * N * 8}))
        return

    def build(dtype):
        H = chf.levels_create(A)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for ps, basis in zip(pro, bases):
            chf.levels_add_coarse(H, ps.shape[1], ps.indptr, ps.indices, ps.data, basis)
        torch.cuda.synchronize()
        t_gal = time.perf_counter() - t
        t = time.perf_counter()
        chf.levels_setup(H, degree=k, pattern=1, tmax=args.tmax, dtype=dtype, v0=v0)
        torch.cuda.synchronize()
        return H, {"galerkin_ms": 1e3 * t_gal, "levels_setup_ms": 1e3 * (time.perf_counter() - t)}

    log("set-up FP64 hierarchy (adaptive pattern, FSAI, Lanczos, coarse inverse)")
    H, setup64 = build(chf.F64)
    setup64 = {"bsr_create_ms": bsr_create_ms, **setup64}
    # the level-0 pattern alone, timed
    torch.cuda.synchronize()
    t = time.perf_counter()
    P0 = chf.pattern_adaptive(A, args.tmax)
    t_pat = time.perf_counter() - t
    rp, _ = chf.pattern_export(P0)
    nnzg = int(rp[-1])
    t = time.perf_counter()
    Gtmp = chf.fsai_setup(A, P0)
    torch.cuda.synchronize()
    t_fsai = time.perf_counter() - t
    del Gtmp
    _, G0, _ = chf.levels_get(H, 0)
    beta0 = chf.levels_get_beta(H, 0)
    # the level-0 spectral bound alone (100 Lanczos steps on G A G^T), timed
    torch.cuda.synchronize()
    t = time.perf_counter()
    chf.lmax_lanczos(A, G0, v0[0])
    t_lz = time.perf_counter() - t
    setup64.update({"adaptive_pattern_level0_ms": 1e3 * t_pat, "fsai_setup_level0_ms": 1e3 * t_fsai,
                     "lanczos_level0_ms": 1e3 * t_lz})
    log(f"set-up done: {setup64}")
    N = A.info()[0] * b

    # ---- timed region: K smoother applications on level 0 (x != 0)
    stream = torch.cuda.current_stream()
    x = torch.zeros(N, dtype=torch.float64, device=dev)
    work = torch.zeros(3 * N, dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        chf.cheb4_smooth(A, G0, beta0, k, bd, x, x_is_zero=False, work=work)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        chf.cheb4_smooth(A, G0, beta0, k, bd, x, x_is_zero=False, work=work)
    e1.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    ms_app = e0.elapsed_time(e1) / args.steps
    gdofs = N * k / (ms_app * 1e-3) / 1e9
    s = 8
    b_step = nnzb * (b * b * s + 4) + 2 * nnzg * (b * b * s + 4) + 10 * N * s
    b_app = k * b_step
    log(f"smoother: {ms_app:.3f} ms/application, {gdofs:.3f} GDOF/s, "
        f"{b_app / (ms_app * 1e-3) / 1e9:.0f} GB/s algorithmic")

    # the same application timed call by call (median of 20 event pairs), with
    # x != 0 and with x0 = 0 (one product with A and 5 N vector values fewer)
    def median_ms(x_is_zero, reps=20):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for _ in range(3):
            chf.cheb4_smooth(A, G0, beta0, k, bd, x, x_is_zero=x_is_zero, work=work)
        for a_, b_ in evs:
            a_.record(stream)
            chf.cheb4_smooth(A, G0, beta0, k, bd, x, x_is_zero=x_is_zero, work=work)
            b_.record(stream)
        torch.cuda.synchronize()
        return float(np.median([a_.elapsed_time(b_) for a_, b_ in evs]))
    med_x = median_ms(False)
    med_0 = median_ms(True)
    b_app0 = b_app - (nnzb * (b * b * s + 4) + 5 * N * s)
    log(f"smoother medians: x != 0 {med_x:.3f} ms, x0 = 0 {med_0:.3f} ms")

    # ---- dominant kernel: the A residual SpMV r = b - A x, timed alone
    r = torch.empty_like(x)
    for _ in range(3):
        chf.bsr_spmv(A, x, r, bvec=bd)
    torch.cuda.synchronize()
    reps = max(20, args.steps)
    e0.record(stream)
    for _ in range(reps):
        chf.bsr_spmv(A, x, r, bvec=bd)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_k1 = e0.elapsed_time(e1) / reps
    bytes_k1 = nnzb * (b * b * 8 + 4) + 3 * N * 8
    achieved = bytes_k1 / (ms_k1 * 1e-3) / 1e9
    log(f"residual SpMV: {ms_k1:.4f} ms, {achieved:.0f} GB/s algorithmic")

    out = {
        "metric": "smoother GDOF/s (%HBM peak) + PCG time to 1e-8, FP64 vs mixed, 1 GPU",
        "value": round(gdofs, 4),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_app, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"biharmonic-like 2D PUM-shaped A=R^T(L^2 (x) I_b)R, {n}x{n} patches, b={b}, "
                         f"{N} dofs, adaptive block-FSAI t_max={args.tmax}, fourth-kind Chebyshev degree {k}, "
                         f"{L}-level Galerkin V({k},{k}) PCG, bilinear patch transfer with Dirichlet nodes, "
                         f"finest transfer P = R^-1 (P_s (x) I_b)"),
            "patches": n, "block": b, "ndof": N, "nnzb_A": nnzb, "nnzb_G": nnzg, "degree": k,
            "tmax": args.tmax, "levels": L, "rhs": "N(0,1) seed 0",
        },
        "smoother": {
            "ms_per_application": round(ms_app, 5),
            "algorithmic_bytes_per_application": b_app,
            "achieved_GBs": round(b_app / (ms_app * 1e-3) / 1e9, 1),
            "hbm_frac": round(b_app / (ms_app * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "wall_s_timed_region": round(t_wall, 4),
            "median_ms_per_application_20_calls": round(med_x, 5),
            "median_hbm_frac": round(b_app / (med_x * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "x0_zero": {"median_ms_per_application_20_calls": round(med_0, 5),
                        "algorithmic_bytes_per_application": b_app0,
                        "hbm_frac": round(b_app0 / (med_0 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        },
        "roofline": {
            "kernel": "k_sell_spmv<10,double,double,EPI_RES> (r = b - A x, level 0)",
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
            "avg_launch_ms": round(ms_k1, 5), "algorithmic_bytes_per_launch": bytes_k1,
            "rocprof_avg_launch_ms": rocprof_residual_avg_ms(),
            "rocprof_frac": (round(bytes_k1 / (rocprof_residual_avg_ms() * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                             if rocprof_residual_avg_ms() else None),
        },
        "setup_fp64": {kk: round(v, 2) for kk, v in setup64.items()},
    }

    # ---- PCG FP64 and mixed
    if not args.no_pcg:
        res = {}
        for name, dt, flex, Hh in [("fp64", chf.F64, False, H), ("mixed_f32", chf.F32, True, None),
                                   ("mixed_bf16g", chf.BF16, True, None), ("fp64_bf16g", chf.F64_BF16G, False, None)]:
            setup = None
            if Hh is None:
                log(f"set-up {name} hierarchy")
                Hh, setup = build(dt)
            xs = torch.zeros(N, dtype=torch.float64, device=dev)
            chf.pcg_solve(Hh, bd, xs, rtol=1e-8, maxit=200, flexible=flex)   # warm-up
            torch.cuda.synchronize()
            t = time.perf_counter()
            it, hist, tr, rc = chf.pcg_solve(Hh, bd, xs, rtol=1e-8, maxit=200, flexible=flex,
                                             raise_on_noconv=False)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            res[name] = {"iterations": it, "time_ms": round(1e3 * el, 2), "ms_per_iteration": round(1e3 * el / max(it, 1), 3),
                         "final_relres": float(hist[-1]), "true_relres": tr, "converged": rc == 0,
                         "flexible_cg": flex}
            if setup:
                res[name]["setup"] = {kk: round(v, 2) for kk, v in setup.items()}
            if dt != chf.F64:
                # one level-0 smoother application with this hierarchy's operators
                # (A in FP32, G in FP32 or BF16, FP32 vectors; or FP64 A and vectors
                # with BF16 G), timed like the FP64 one
                A0m, G0m, _ = chf.levels_get(Hh, 0)
                beta_m = chf.levels_get_beta(Hh, 0)
                vt = torch.float64 if dt == chf.F64_BF16G else torch.float32
                b32 = bd.to(vt)
                x32 = torch.zeros(N, dtype=vt, device=dev)
                w32 = torch.zeros(3 * N, dtype=vt, device=dev)
                for _ in range(args.warmup):
                    chf.cheb4_smooth(A0m, G0m, beta_m, k, b32, x32, work=w32, dtype=dt)
                torch.cuda.synchronize()
                e0.record(stream)
                for _ in range(args.steps):
                    chf.cheb4_smooth(A0m, G0m, beta_m, k, b32, x32, work=w32, dtype=dt)
                e1.record(stream)
                torch.cuda.synchronize()
                ms_m = e0.elapsed_time(e1) / args.steps
                sg = 4 if dt == chf.F32 else 2
                sa = sv = 8 if dt == chf.F64_BF16G else 4
                b_m = k * (nnzb * (b * b * sa + 4) + 2 * nnzg * (b * b * sg + 4) + 10 * N * sv)
                res[name]["smoother"] = {"ms_per_application": round(ms_m, 5), "algorithmic_bytes_per_application": b_m,
                                         "achieved_GBs": round(b_m / (ms_m * 1e-3) / 1e9, 1),
                                         "hbm_frac": round(b_m / (ms_m * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            log(f"PCG {name}: {res[name]}")
            if Hh is not H:
                Hh.destroy()
        if n == 512 and L == 6 and k == 4 and args.tmax == 8 and os.path.exists(GOLDEN_C1):
            gold = json.load(open(GOLDEN_C1))["dirichlet"]["pcg"]
            for name in ("fp64", "mixed_f32", "mixed_bf16g", "fp64_bf16g"):
                if name in gold:
                    res[name]["oracle_iterations"] = gold[name]["iterations"]
        res["mixed_f32_over_fp64_time"] = round(res["mixed_f32"]["time_ms"] / res["fp64"]["time_ms"], 4)
        res["mixed_bf16g_over_fp64_time"] = round(res["mixed_bf16g"]["time_ms"] / res["fp64"]["time_ms"], 4)
        res["fp64_bf16g_over_fp64_time"] = round(res["fp64_bf16g"]["time_ms"] / res["fp64"]["time_ms"], 4)
        out["pcg"] = res

    if not args.no_comparators:
        out["comparators"] = comparators_leg(args, chf, torch, dev, H, A, bd, N, k)
    if not args.no_nested:
        out["nested"] = nested_leg(args, chf, torch, dev, A, bd, N, k, pro, bases, v0, H,
                                   setup64["levels_setup_ms"])
    if not args.no_learned:
        out["learned"] = learned_leg(args, chf, torch, dev, n, b, L, k, pro, bases)
    if not args.no_setup3d:
        out["setup3d"] = setup3d_leg(args, chf, torch)
    if not args.no_c2:
        out["c2"] = c2_leg(args, chf, torch, dev)

    if not args.no_cpu_baseline:
        log("timing the oracle on the host")
        out["cpu_baseline"] = cpu_baseline(args.cpu_grid, b, args.tmax, k)
        if not args.no_setup3d:
            out["cpu_baseline"]["oracle_setup3d_sampled"] = cpu_setup3d_sample(args.setup3d_grid, b,
                                                                               args.setup3d_tmax)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
