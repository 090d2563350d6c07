"""Shared helpers for the GPU tests: upload seeded inputs through the C ABI
binding and compare against the oracle."""
import numpy as np

from problems import grid_sizes, lanczos_starts, level_basis, make_problem, prolongator


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    scale = np.abs(want).max()
    return float(np.abs(got - want).max() / (scale if scale > 0 else 1.0))


def dev(x, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda")


def host(t):
    return t.detach().to("cpu").numpy()


def upload(p):
    import paper_2509_06744_amd as chf
    return chf.bsr_create(p.nb, p.b, p.rowptr, p.colidx, p.vals)


def hierarchy_inputs(n, dim, b, levels, seed, order=2):
    """Prolongators (finest first) and Lanczos start vectors for each level;
    order: interpolation nodes per direction of the patch transfer."""
    sizes = grid_sizes(n, levels)
    pro = [prolongator(sizes[l + 1], dim, order) for l in range(levels - 1)]
    starts = lanczos_starts(seed, [s ** dim * b for s in sizes])
    return pro, starts


def oracle_levels(p, levels, mode="lower", tmax=0, seed=0, order=2, **kw):
    from oracle import solver
    from oracle.bsr import from_problem
    pro, starts = hierarchy_inputs(p.n, p.dim, p.b, levels, seed, order)
    return solver.build_levels(from_problem(p), pro, starts, mode, tmax, bases=level_basis(p, levels), **kw)


def gpu_levels(p, levels, degree, pattern, tmax=0, dtype=0, seed=0, betas=None, level0_pattern=None, order=2):
    """Build the GPU hierarchy for problem p through the C ABI."""
    import paper_2509_06744_amd as chf
    A = upload(p)
    pro, starts = hierarchy_inputs(p.n, p.dim, p.b, levels, seed, order)
    L = chf.levels_create(A)
    for ps, basis in zip(pro, level_basis(p, levels)):
        ps = ps.tocsr()
        chf.levels_add_coarse(L, ps.shape[1], ps.indptr, ps.indices, ps.data, basis)
    v0 = None if betas is not None else [dev(s) for s in starts[:-1]]
    if level0_pattern is not None:
        chf.levels_set_pattern(L, 0, level0_pattern)
    chf.levels_setup(L, degree=degree, pattern=pattern, tmax=tmax, dtype=dtype, v0=v0)
    if betas is not None:
        for l, bt in enumerate(betas):
            chf.levels_set_beta(L, l, bt)
    return A, L, pro, starts
