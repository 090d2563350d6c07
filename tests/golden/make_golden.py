"""Writes the stored oracle results under tests/golden/ from the oracle alone.

--workload c1 (tests/golden/c1_pcg_iterations.json): biharmonic-like 2D
problem on 512 x 512 patches, b = 10, seed 0 (A = R^T (L^2 (x) I_b) R),
six-level Galerkin hierarchy with the bilinear patch transfer (--boundary
dirichlet, the default: Lagrange interpolation with the Dirichlet boundary
points as nodes; --boundary zero_ghost: the earlier reading with zero ghost
cells), PCG to a recursive relative residual of 1e-8.

--workload c2 (tests/golden/c2_n<N>_pcg_iterations.json): triharmonic-like
2D problem (D = L^3) on N x N patches (default 32), b = 21, seed 0, three
levels, cubic patch transfer with the Dirichlet boundary points as nodes,
PCG to a recursive relative residual of 1e-10.

Both: adaptive block-FSAI on every smoothed level (Algorithm 1, P0 =
diagonal, tau = 1, t_max = 8), Lanczos bounds (Sec. 5: 100 steps, x 1.01),
V(4,4) with fourth-kind Chebyshev smoothing, PCG from x = 0 in four forms:
FP64 (Fletcher-Reeves), the mixed forms with A, G in FP32 or A in FP32 and G
in BF16 (flexible PCG around the FP32 cycle), and FP64 with G rounded to BF16
(Fletcher-Reeves).

Only oracle/ and the input generator are called. Block rows are independent
in Algorithm 1 and in the factor of Def. 2.2, so their rows are computed by a
pool of worker processes, each running the oracle's own per-row functions on
a contiguous chunk of rows; the results are the same as one serial pass.
Run from the repository root:  python tests/golden/make_golden.py
(c1: about an hour on 8 cores; --n 64 gives a quick smaller c1 run written
to _work/ instead of the golden file).
"""
from __future__ import annotations

import os

# one BLAS thread per worker process: the pool supplies the parallelism
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"

import argparse
import hashlib
import json
import multiprocessing as mp
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import adaptive, fsai, lanczos, mixed, multilevel  # noqa: E402
from oracle.bsr import Bsr, from_problem  # noqa: E402
from problems import grid_sizes, lanczos_starts, level_basis, make_problem, prolongator, rhs  # noqa: E402

_A = None   # the level operator shared with the forked workers


def _pattern_chunk(args):
    lo, hi, tmax = args
    return adaptive.adaptive_pattern(_A, tmax, 1.0, rows=range(lo, hi))


def _fsai_chunk(args):
    lo, hi, prow, pcol = args
    return fsai.fsai_rows(_A, range(lo, hi), prow, pcol)


def _chunks(n, parts):
    step = max(1, (n + parts - 1) // parts)
    return [(s, min(n, s + step)) for s in range(0, n, step)]


def pattern_hash(prow, pcol) -> str:
    h = hashlib.sha256()
    h.update(np.asarray(prow, dtype=np.int64).tobytes())
    h.update(np.asarray(pcol, dtype=np.int64).tobytes())
    return h.hexdigest()


def log(msg):
    print(f"[golden {time.strftime('%H:%M:%S')}] {msg}", flush=True)


def build(a0: Bsr, pro, bases, starts, tmax, workers):
    global _A
    levels = []
    a = a0
    nl = len(pro) + 1
    info = []
    for l in range(nl):
        lev = multilevel.Level(a=a)
        if l == nl - 1:
            lev.finish()
            lev.chol = multilevel.coarse_factor(a)
            levels.append(lev)
            break
        _A = a      # forked workers see this level's operator
        pool = mp.get_context("fork").Pool(workers)
        t0 = time.time()
        parts = pool.map(_pattern_chunk, [(lo, hi, tmax) for lo, hi in _chunks(a.nb, 16 * workers)])
        prow, pcol = [0], []
        for pr, pc in parts:
            pcol.extend(pc.tolist())
            prow.extend((prow[-1] + pr[1:]).tolist())
        prow = np.array(prow, dtype=np.int64)
        pcol = np.array(pcol, dtype=np.int64)
        fsai.check_pattern(a.nb, prow, pcol)
        t1 = time.time()
        rows = pool.map(_fsai_chunk, [(lo, hi, prow, pcol) for lo, hi in _chunks(a.nb, 16 * workers)])
        pool.close()
        pool.join()
        gvals = np.zeros((len(pcol), a.b, a.b))
        for d in rows:
            for k, blocks in d.items():
                gvals[prow[k]:prow[k + 1]] = blocks
        lev.g = Bsr(prow, pcol, gvals, a.b)
        t2 = time.time()
        lev.p_s = pro[l]
        lev.basis = bases[l]
        lev.finish()
        lev.beta, theta = lanczos.lmax(lev.apply_b, np.asarray(starts[l]), 100, 1.01)
        t3 = time.time()
        info.append({"level": l, "nb": int(a.nb), "nnzb_A": int(a.nnzb), "nnzb_G": int(len(pcol)),
                     "pattern_sha256": pattern_hash(prow, pcol), "beta": lev.beta, "theta": theta})
        log(f"level {l}: nb {a.nb}, G blocks {len(pcol)}, pattern {t1 - t0:.0f} s, factor {t2 - t1:.0f} s, "
            f"Lanczos {t3 - t2:.0f} s, beta {lev.beta:.6f}")
        levels.append(lev)
        a = multilevel.galerkin(a, pro[l], bases[l])
        log(f"level {l + 1} Galerkin: nb {a.nb}, blocks {a.nnzb}")
    return levels, info


def run_pcg(name, apply_a, prec, bvec, flexible, rtol=1e-8, maxit=300):
    t0 = time.time()
    _, it, hist, tr = multilevel.pcg(apply_a, prec, bvec, rtol, maxit, flexible=flexible)
    rec = {"iterations": it, "final_relres": hist[-1], "true_relres": tr, "flexible": flexible,
           "oracle_seconds": round(time.time() - t0, 1)}
    log(f"PCG {name}: {rec}")
    return rec


_PCG = None   # (levels, starts, bvec, k), shared with the forked PCG workers


def _pcg_worker(form):
    levels, starts, bvec, k, rtol = _PCG
    if form == "fp64":
        return form, run_pcg(form, levels[0].apply_a, lambda r: multilevel.vcycle(levels, 0, r, k), bvec, False,
                             rtol), None
    if form == "fp64_bf16g":
        lb = mixed.bf16g_levels(levels, starts)
        return form, run_pcg(form, levels[0].apply_a, lambda r: multilevel.vcycle(lb, 0, r, k), bvec, False,
                             rtol), [m.beta for m in lb[:-1]]
    ml = mixed.mixed_levels(levels, "f32" if form == "mixed_f32" else "bf16", starts)
    betas = [m.beta for m in ml[:-1]]
    return form, run_pcg(form, levels[0].apply_a, mixed.precond_mixed(ml, k), bvec, True, rtol), betas


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c1", choices=["c1", "c2"])
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--levels", type=int, default=None)
    ap.add_argument("--workers", type=int, default=max(1, min(8, os.cpu_count() or 1) - 1))
    ap.add_argument("--boundary", default="dirichlet", choices=["dirichlet", "zero_ghost"])
    args = ap.parse_args()
    c1 = args.workload == "c1"
    n = args.n or (512 if c1 else 32)
    nl = args.levels or (6 if c1 else 3)
    b, power, order, rtol = (10, 2, 2, 1e-8) if c1 else (21, 3, 4, 1e-10)
    tmax, k = 8, 4
    p = make_problem(n, 2, b, power, seed=0)
    sizes = grid_sizes(n, nl)
    pro = [prolongator(sizes[l + 1], 2, order, args.boundary) for l in range(nl - 1)]
    starts = lanczos_starts(0, [s * s * b for s in sizes])
    bases = level_basis(p, nl)
    bvec = rhs(0, p.ndof)
    ctx = mp.get_context("fork")
    t0 = time.time()
    levels, info = build(from_problem(p), pro, bases, starts, tmax, args.workers)
    log(f"hierarchy built in {time.time() - t0:.0f} s")
    out = {"workload": f"{'biharmonic' if c1 else 'triharmonic'}-like 2D, {n}x{n} patches, b={b}, seed 0, "
                       f"{nl} levels, {'bilinear' if order == 2 else 'cubic'} transfer ({args.boundary} boundary), "
                       f"adaptive t_max={tmax}, V({k},{k}) fourth-kind Chebyshev, PCG rtol {rtol:g}",
           "levels": info, "pcg": {}}
    global _PCG
    _PCG = (levels, starts, bvec, k, rtol)   # forked workers read it; only the form name is sent
    with ctx.Pool(4) as pool:
        for form, rec, betas in pool.imap_unordered(_pcg_worker, ["fp64", "mixed_f32", "mixed_bf16g", "fp64_bf16g"]):
            if betas is not None:
                rec["betas"] = betas
            out["pcg"][form] = rec
    if c1:
        path = (os.path.join(ROOT, "tests", "golden", "c1_pcg_iterations.json") if n == 512 and nl == 6
                else os.path.join(ROOT, "_work", f"golden_n{n}_l{nl}.json"))
    else:
        path = os.path.join(ROOT, "tests", "golden", f"c2_n{n}_pcg_iterations.json")
    os.makedirs(os.path.dirname(path), exist_ok=True)
    allrec = {}
    if os.path.exists(path):
        with open(path) as f:
            allrec = json.load(f)
    allrec[args.boundary] = out
    with open(path, "w") as f:
        json.dump(allrec, f, indent=1)
    log(f"wrote {path} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
