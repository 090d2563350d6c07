"""Seeded synthetic inputs shaped like partition-of-unity (PUM) discretisations.

This package produces *inputs only*: block-sparse SPD matrices, right-hand
sides, prolongation weights and the random start vectors that the method
consumes. It holds none of the method's arithmetic (no FSAI, no smoother, no
Galerkin product, no Krylov iteration), so both the oracle and the HIP path may
use it.
"""
from .generator import (  # noqa: F401
    Problem,
    VarProblem,
    make_vb_problem,
    vb_block_sizes,
    laplacian,
    stencil_matrix,
    make_problem,
    prolongator_1d,
    prolongator,
    level_basis,
    rhs,
    lanczos_starts,
    uniform_start,
    grid_sizes,
    mlp_init,
    permutation,
)
from .configs import CONFIGS, ProblemConfig  # noqa: F401
