"""The allocation-free smoother entry point (chf_cheb4_smooth_noalloc, work
vectors in the library's static device array) against chf_cheb4_smooth with a
caller-provided work buffer: same kernels, same order, so the outputs must be
bit-identical. Two calls in a row on different problems (the second smaller),
FP64 and FP32 storage, the size limit and the FP32-layout precondition."""
import numpy as np
import pytest

from problems import make_problem, rhs
from tests.helpers import dev, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def chf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    import paper_2509_06744_amd as m
    m.lib()
    return m


def _case(chf, n, b, store, x_is_zero, seed):
    import torch
    p = make_problem(n, 2, b, 2, seed=seed)
    A = upload(p)
    G = chf.fsai_setup(A, chf.pattern_lower(A), g_store=store)
    vt = torch.float64 if store == chf.F64 else torch.float32
    beta = 2.0
    bvec = dev(rhs(seed, p.ndof), vt)
    x0 = dev(np.random.default_rng(seed + 1).standard_normal(p.ndof), vt)
    return p, A, G, vt, beta, bvec, x0


@pytest.mark.parametrize("x_is_zero", [True, False])
def test_noalloc_matches_work_buffer_fp64_two_calls(chf, x_is_zero):
    import torch
    for n, b, deg in [(48, 10, 4), (20, 3, 3)]:          # second call on a smaller problem
        p, A, G, vt, beta, bvec, x0 = _case(chf, n, b, chf.F64, x_is_zero, n)
        x_ref = x0.clone()
        work = torch.full((3 * p.ndof,), float("nan"), dtype=vt, device="cuda")
        chf.cheb4_smooth(A, G, beta, deg, bvec, x_ref, x_is_zero=x_is_zero, work=work)
        x = x0.clone()
        chf.cheb4_smooth_noalloc(A, G, beta, deg, bvec, x, x_is_zero=x_is_zero)
        torch.cuda.synchronize()
        assert torch.isfinite(x).all()
        assert torch.equal(x, x_ref), (n, b)


def test_noalloc_fp32_needs_layout_then_matches(chf):
    import torch
    for n, b in [(40, 10), (16, 3)]:
        p, A, G, vt, beta, bvec, x0 = _case(chf, n, b, chf.F32, False, n)
        with pytest.raises(chf.ChfError) as ei:
            chf.cheb4_smooth_noalloc(A, G, beta, 4, bvec, x0.clone(), dtype=chf.F32)
        assert ei.value.code == -1
        x_ref = x0.clone()
        work = torch.zeros(3 * p.ndof, dtype=vt, device="cuda")
        chf.cheb4_smooth(A, G, beta, 4, bvec, x_ref, work=work, dtype=chf.F32)   # builds A's FP32 layout
        x = x0.clone()
        chf.cheb4_smooth_noalloc(A, G, beta, 4, bvec, x, dtype=chf.F32)
        torch.cuda.synchronize()
        assert torch.equal(x, x_ref)


def test_noalloc_rejects_sizes_past_the_scratch(chf):
    import torch
    nb = 2796203                     # 3 * nb * 8 bytes is just past 64 MiB
    rowptr = np.arange(nb + 1, dtype=np.int64)
    cols = np.arange(nb, dtype=np.int32)
    A = chf.bsr_create(nb, 1, rowptr, cols, np.ones(nb))
    G = chf.fsai_setup(A, chf.pattern_from_csr(nb, rowptr, cols))
    bvec = torch.ones(nb, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(bvec)
    with pytest.raises(chf.ChfError) as ei:
        chf.cheb4_smooth_noalloc(A, G, 1.5, 2, bvec, x, x_is_zero=True)
    assert ei.value.code == -1
    # one row fewer fits
    rowptr2 = np.arange(nb, dtype=np.int64)
    A2 = chf.bsr_create(nb - 1, 1, rowptr2, cols[:-1], np.ones(nb - 1))
    G2 = chf.fsai_setup(A2, chf.pattern_from_csr(nb - 1, rowptr2, cols[:-1]))
    b2 = torch.ones(nb - 1, dtype=torch.float64, device="cuda")
    x2 = torch.zeros_like(b2)
    chf.cheb4_smooth_noalloc(A2, G2, 1.5, 2, b2, x2, x_is_zero=True)
    # A = I, M = I: degree 2 on [0, 1.5] gives x = (1 - W^_2(1)) b, W^_2 from Eq. chebyshev_4th_kind
    t = 1.0 - 2.0 / 1.5
    w2 = (4 * t * t + 2 * t - 1) / 5.0
    torch.cuda.synchronize()
    assert torch.allclose(x2, torch.full_like(x2, 1.0 - w2), rtol=1e-14, atol=0)
