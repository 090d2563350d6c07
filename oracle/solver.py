"""Hierarchy set-up for the oracle: Galerkin levels, one block-FSAI factor and
one Lanczos bound per level, dense Cholesky on the coarsest level."""
from __future__ import annotations

import numpy as np

from . import adaptive, fsai, lanczos, nested
from .bsr import Bsr
from .multilevel import Level, coarse_factor, galerkin


def make_pattern(a: Bsr, mode: str, tmax: int = 0, tau: float = 1.0):
    if mode == "lower":
        return fsai.pattern_lower(a)
    if mode == "adaptive":
        return adaptive.adaptive_pattern(a, tmax, tau)
    if mode == "diagonal":
        return fsai.pattern_diagonal(a.nb)
    raise ValueError(mode)


def build_levels(a0: Bsr, prolongators, starts, mode: str, tmax: int = 0,
                 tau: float = 1.0, iters: int = 100, safety: float = 1.01,
                 patterns=None, betas=None, bases=None, nest: bool = False):
    """prolongators[l] maps level l+1 to level l (scalar patch weights, with
    the block-diagonal basis change bases[l] when given: P = T (P_s (x) I));
    starts[l] is the Lanczos start vector of level l. ``patterns``/``betas``
    may fix the per-level pattern or bound instead of computing them.
    nest: nested block-FSAI with one level (Sec. 2.2) on every smoothed level,
    the inner pattern from Algorithm 1 with the same t_max and tau."""
    levels = []
    a = a0
    nl = len(prolongators) + 1
    for l in range(nl):
        lev = Level(a=a)
        if l < nl - 1:
            prow, pcol = patterns[l] if patterns is not None else make_pattern(a, mode, tmax, tau)
            if nest:
                lev.g, _, _, lev.g1 = nested.nested(a, (prow, pcol), tmax, tau)
            else:
                lev.g = fsai.fsai(a, prow, pcol)
            lev.p_s = prolongators[l]
            lev.basis = bases[l] if bases is not None else None
            lev.finish()
            if betas is not None:
                lev.beta = betas[l]
            else:
                lev.beta, _ = lanczos.lmax(lev.apply_b, np.asarray(starts[l]), iters, safety)
            a = galerkin(a, prolongators[l], lev.basis)
        else:
            lev.finish()
            lev.chol = coarse_factor(a)
        levels.append(lev)
    return levels
