"""chf_pattern_template (host code of the C library, no GPU needed): rows
built from a stencil template, against a direct construction; rejection of
offsets that do not point to smaller indices; and the translation invariance
it relies on: the template read off one interior row of Algorithm 1's pattern
(the oracle, on the scalar biharmonic-like D) reproduces Algorithm 1 on every
row far enough from the boundary."""
import numpy as np
import pytest

from oracle import adaptive
from oracle.bsr import from_problem
from problems import make_problem


def _direct(nx, ny, nz, offs):
    rowptr, cols = [0], []
    for k in range(nx * ny * nz):
        kx, ky, kz = k % nx, (k // nx) % ny, k // (nx * ny)
        row = set()
        for dx, dy, dz in offs:
            cx, cy, cz = kx + dx, ky + dy, kz + dz
            if 0 <= cx < nx and 0 <= cy < ny and 0 <= cz < nz:
                row.add(cx + nx * (cy + ny * cz))
        cols.extend(sorted(row) + [k])
        rowptr.append(len(cols))
    return np.array(rowptr), np.array(cols)


def test_template_matches_direct_construction():
    import paper_2509_06744_amd as chf
    offs = [(-1, 0, 0), (0, -1, 0), (2, -1, 0), (-3, 1, -1), (0, 0, -2), (-1, -1, 0)]
    P = chf.pattern_template(7, 5, 3, offs)
    rp, cp = chf.pattern_export(P)
    wr, wc = _direct(7, 5, 3, offs)
    assert np.array_equal(rp, wr) and np.array_equal(cp, wc)


def test_template_rejects_offsets_to_larger_indices():
    import paper_2509_06744_amd as chf
    with pytest.raises(chf.ChfError) as ei:
        chf.pattern_template(6, 6, 1, [(-1, 0, 0), (1, 0, 0)])
    assert ei.value.code == -1


def test_interior_template_reproduces_algorithm1():
    import paper_2509_06744_amd as chf
    from paper_2509_06744_amd import learned
    n, tmax = 16, 8
    a = from_problem(make_problem(n, 2, 1, 2, seed=0, rotate=False))
    prow, pcol = adaptive.adaptive_pattern(a, tmax)
    k0 = (n // 2) * n + n // 2
    offs = learned.template_offsets(prow, pcol, n, n, k0)
    assert len(offs) == tmax
    P = chf.pattern_template(n, n, 1, offs)
    rp, cp = chf.pattern_export(P)
    reach = 4          # rows this far from every edge see no boundary in t_max steps
    inner = [k for k in range(n * n) if reach <= k % n < n - reach and reach <= k // n < n - reach]
    for k in inner:
        assert np.array_equal(cp[rp[k]:rp[k + 1]], pcol[prow[k]:prow[k + 1]]), k
    # near the boundary the template is only an approximation
    assert any(not np.array_equal(cp[rp[k]:rp[k + 1]], pcol[prow[k]:prow[k + 1]]) for k in range(n * n))
