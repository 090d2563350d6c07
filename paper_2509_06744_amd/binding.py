"""ctypes marshalling for the C ABI in include/chf.h."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

__all__ = [
    "F64", "F32", "BF16", "F64_BF16G", "NFEAT", "NPARAM", "SMOOTH_CHEB4", "SMOOTH_CHEB1", "SMOOTH_RICHARDSON", "CYCLE_VKK", "CYCLE_V2K0",
    "ChfError", "lib", "lib_path", "version", "current_stream",
    "Bsr", "Pattern", "Fsai", "Levels", "Mlp", "LevelOpts",
    "bsr_create", "bsr_export", "bsr_spmv", "vbsr_create", "vbsr_info",
    "pattern_lower", "pattern_from_csr", "pattern_adaptive", "pattern_template", "pattern_export",
    "fsai_setup", "fsai_export", "fsai_export_flat", "fsai_apply", "bsr_triple", "fsai_nest", "lmax_lanczos",
    "cheb4_smooth", "cheb4_smooth_noalloc", "cheb1_smooth", "richardson_smooth",
    "levels_create", "levels_add_coarse", "levels_setup", "levels_get", "levels_get_beta",
    "levels_set_beta", "levels_set_cycle", "levels_set_nesting", "levels_info", "levels_set_pattern", "vcycle", "pcg_solve",
    "levels_energy_factor",
    "bicgstab_solve",
    "mlp_candidates", "mlp_features", "mlp_create", "mlp_get_params", "mlp_forward",
    "mlp_loss_grad", "mlp_train_step", "mlp_propose", "mlp_labels", "mlp_train",
    "EXPORTED",
]

F64, F32, BF16, F64_BF16G = 0, 1, 2, 3
SMOOTH_CHEB4, SMOOTH_CHEB1, SMOOTH_RICHARDSON = 0, 1, 2
CYCLE_VKK, CYCLE_V2K0 = 0, 1
CHF_ENOCONV = -5
NFEAT, NPARAM = 6, 4673   # learned proposer: features per candidate, network parameters

HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(HERE, "libchf.so")

# every entry point declared in include/chf.h: (restype, argtypes)
_vp, _i32, _i64, _dbl, _flt = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_float
_pi64, _pi32, _pd, _pf, _pint = (C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                 C.POINTER(C.c_float), C.POINTER(C.c_int))


class LevelOpts(C.Structure):
    _fields_ = [("degree", C.c_int), ("pattern", C.c_int), ("tmax", C.c_int), ("tau", C.c_double),
                ("lanczos_iters", C.c_int), ("safety", C.c_double), ("dtype", C.c_int)]


EXPORTED = {
    "chf_last_error": (C.c_char_p, []),
    "chf_version": (C.c_char_p, []),
    "chf_bsr_create": (C.c_int, [_i64, _i32, _vp, _vp, _vp, C.c_int, C.POINTER(_vp)]),
    "chf_bsr_destroy": (C.c_int, [_vp]),
    "chf_vbsr_create": (C.c_int, [_i64, _vp, _vp, _vp, _vp, C.POINTER(_vp)]),
    "chf_vbsr_info": (C.c_int, [_vp, _pi64, _pi64, _vp]),
    "chf_bsr_info": (C.c_int, [_vp, _pi64, _pi32, _pi64]),
    "chf_bsr_export": (C.c_int, [_vp, _vp, _vp, _vp]),
    "chf_bsr_spmv": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, C.c_int, _vp]),
    "chf_pattern_lower": (C.c_int, [_vp, C.POINTER(_vp)]),
    "chf_pattern_from_csr": (C.c_int, [_i64, _vp, _vp, C.POINTER(_vp)]),
    "chf_pattern_adaptive": (C.c_int, [_vp, _vp, C.c_int, _dbl, C.POINTER(_vp)]),
    "chf_pattern_template": (C.c_int, [_i64, _i64, _i64, _i32, _vp, C.POINTER(_vp)]),
    "chf_pattern_info": (C.c_int, [_vp, _pi64, _pi64]),
    "chf_pattern_export": (C.c_int, [_vp, _vp, _vp]),
    "chf_pattern_destroy": (C.c_int, [_vp]),
    "chf_fsai_setup": (C.c_int, [_vp, _vp, C.c_int, C.POINTER(_vp), _pi64]),
    "chf_fsai_destroy": (C.c_int, [_vp]),
    "chf_fsai_export": (C.c_int, [_vp, _vp]),
    "chf_fsai_apply": (C.c_int, [_vp, C.c_int, _vp, _vp, _vp, _vp]),
    "chf_lmax_lanczos": (C.c_int, [_vp, _vp, C.c_int, C.c_int, _vp, _dbl, _pd, _pd, _vp]),
    "chf_cheb4_smooth": (C.c_int, [_vp, _vp, C.c_int, _dbl, C.c_int, _vp, _vp, C.c_int, _vp, _vp]),
    "chf_cheb4_smooth_noalloc": (C.c_int, [_vp, _vp, C.c_int, _dbl, C.c_int, _vp, _vp, C.c_int, _vp]),
    "chf_cheb1_smooth": (C.c_int, [_vp, _vp, C.c_int, _dbl, _dbl, C.c_int, _vp, _vp, C.c_int, _vp, _vp]),
    "chf_richardson_smooth": (C.c_int, [_vp, _vp, C.c_int, _dbl, C.c_int, _vp, _vp, C.c_int, _vp, _vp]),
    "chf_levels_set_cycle": (C.c_int, [_vp, C.c_int, _dbl, C.c_int]),
    "chf_bsr_triple": (C.c_int, [_vp, _vp, C.POINTER(_vp)]),
    "chf_levels_set_nesting": (C.c_int, [_vp, C.c_int]),
    "chf_fsai_nest": (C.c_int, [_vp, _vp, C.POINTER(_vp)]),
    "chf_bicgstab_solve": (C.c_int, [_vp, _vp, _vp, _dbl, C.c_int, _pint, _vp, _pd, _vp]),
    "chf_levels_create": (C.c_int, [_vp, C.POINTER(_vp)]),
    "chf_levels_add_coarse": (C.c_int, [_vp, _i64, _vp, _vp, _vp, _vp]),
    "chf_levels_setup": (C.c_int, [_vp, C.POINTER(LevelOpts), C.POINTER(_vp), _pi64]),
    "chf_levels_destroy": (C.c_int, [_vp]),
    "chf_levels_set_pattern": (C.c_int, [_vp, C.c_int, _vp]),
    "chf_levels_info": (C.c_int, [_vp, _pint, _vp]),
    "chf_levels_get": (C.c_int, [_vp, C.c_int, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(_vp)]),
    "chf_levels_get_beta": (C.c_int, [_vp, C.c_int, _pd]),
    "chf_levels_set_beta": (C.c_int, [_vp, C.c_int, _dbl]),
    "chf_vcycle": (C.c_int, [_vp, _vp, _vp, C.c_int, _vp]),
    "chf_pcg_solve": (C.c_int, [_vp, _vp, _vp, _dbl, C.c_int, C.c_int, _pint, _vp, _pd, _vp]),
    "chf_levels_energy_factor": (C.c_int, [_vp, _vp, _dbl, C.c_int, _pd, _pint, _vp]),
    "chf_mlp_candidates": (C.c_int, [_vp, _pi64, _vp, _vp]),
    "chf_mlp_features": (C.c_int, [_vp, _i32, _i32, _vp, _vp]),
    "chf_mlp_create": (C.c_int, [_vp, C.POINTER(_vp)]),
    "chf_mlp_destroy": (C.c_int, [_vp]),
    "chf_mlp_get_params": (C.c_int, [_vp, _vp]),
    "chf_mlp_forward": (C.c_int, [_vp, _vp, _i64, _vp, _vp]),
    "chf_mlp_loss_grad": (C.c_int, [_vp, _vp, _vp, _i64, _pf, _vp, _vp]),
    "chf_mlp_train_step": (C.c_int, [_vp, _vp, _vp, _i64, _flt, _flt, _flt, _flt, _pf, _vp]),
    "chf_mlp_propose": (C.c_int, [_vp, _vp, _i32, _i32, C.c_int, C.POINTER(_vp)]),
    "chf_mlp_labels": (C.c_int, [_vp, _vp, _vp, _vp]),
    "chf_mlp_train": (C.c_int, [_vp, _vp, _vp, _i64, _vp, _i64, C.c_int, _flt, _flt, _flt, _flt, _vp, _vp]),
}

_LIB = None


class ChfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"chf error {code}: {msg}")
        self.code = code


def lib():
    """Load libchf.so (built in-tree by build.py); raises if it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(lib_path):
            raise ImportError(f"{lib_path} is missing: build it with paper_2509_06744_amd/build.py")
        handle = C.CDLL(lib_path)
        for name, (res, args) in EXPORTED.items():
            fn = getattr(handle, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _LIB = handle
    return _LIB


def _fn(name):
    f = getattr(lib(), name, None)
    if f is None:
        raise ImportError(f"{name} is not exported by {lib_path}")
    return f


def _check(rc: int):
    if rc != 0:
        raise ChfError(rc, lib().chf_last_error().decode())


def version() -> str:
    return lib().chf_version().decode()


def current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _host(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def _stream(stream):
    return current_stream() if stream is None else stream


class _Handle:
    _destroy = None

    def __init__(self, h, owner=True):
        self.h = h
        self.owner = owner

    def destroy(self):
        if self.owner and self.h:
            _check(_fn(self._destroy)(self.h))
        self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Bsr(_Handle):
    _destroy = "chf_bsr_destroy"

    def info(self):
        nb, b, nnzb = C.c_int64(), C.c_int32(), C.c_int64()
        _check(_fn("chf_bsr_info")(self.h, C.byref(nb), C.byref(b), C.byref(nnzb)))
        return nb.value, b.value, nnzb.value


class Pattern(_Handle):
    _destroy = "chf_pattern_destroy"


class Fsai(_Handle):
    _destroy = "chf_fsai_destroy"


class Levels(_Handle):
    _destroy = "chf_levels_destroy"


class Mlp(_Handle):
    _destroy = "chf_mlp_destroy"


# ------------------------------------------------------------------- BSR --
def bsr_create(nb, b, rowptr, colidx, vals):
    """vals: host float64 array (nnzb, b, b) or a device float64 torch tensor."""
    rp, rpp = _host(rowptr, np.int64)
    ci, cip = _host(colidx, np.int32)
    on_dev = not isinstance(vals, np.ndarray)
    if on_dev:
        vp = _ptr(vals)
        keep = vals
    else:
        keep, vp = _host(vals, np.float64)
    out = C.c_void_p()
    _check(_fn("chf_bsr_create")(int(nb), int(b), rpp, cip, vp, int(on_dev), C.byref(out)))
    del keep
    return Bsr(out)


def vbsr_create(nb, bsize, rowptr, colidx, vals):
    """Variable block sizes: bsize int32[nb]; vals flat, block by block."""
    bs, bsp = _host(bsize, np.int32)
    rp, rpp = _host(rowptr, np.int64)
    ci, cip = _host(colidx, np.int32)
    vv, vvp = _host(vals, np.float64)
    out = C.c_void_p()
    _check(_fn("chf_vbsr_create")(int(nb), bsp, rpp, cip, vvp, C.byref(out)))
    return Bsr(out)


def vbsr_info(A: Bsr):
    """Returns (unknowns, stored values, block sizes int32[nb])."""
    nb = A.info()[0]
    nd, nv = C.c_int64(), C.c_int64()
    bs = np.empty(nb, np.int32)
    _check(_fn("chf_vbsr_info")(A.h, C.byref(nd), C.byref(nv), bs.ctypes.data_as(C.c_void_p)))
    return nd.value, nv.value, bs


def bsr_export(A: Bsr):
    nb, b, nnzb = A.info()
    rowptr = np.empty(nb + 1, np.int64)
    colidx = np.empty(nnzb, np.int32)
    vals = np.empty((nnzb, b, b), np.float64)
    _check(_fn("chf_bsr_export")(A.h, rowptr.ctypes.data_as(C.c_void_p), colidx.ctypes.data_as(C.c_void_p),
                                 vals.ctypes.data_as(C.c_void_p)))
    return rowptr, colidx, vals


def bsr_spmv(A: Bsr, x, y, bvec=None, dtype=F64, stream=None):
    _check(_fn("chf_bsr_spmv")(A.h, dtype, _ptr(x), _ptr(bvec), _ptr(y), int(bvec is not None), _stream(stream)))


# -------------------------------------------------------------- patterns --
def pattern_lower(A: Bsr) -> Pattern:
    out = C.c_void_p()
    _check(_fn("chf_pattern_lower")(A.h, C.byref(out)))
    return Pattern(out)


def pattern_from_csr(nb, rowptr, colidx) -> Pattern:
    rp, rpp = _host(rowptr, np.int64)
    ci, cip = _host(colidx, np.int32)
    out = C.c_void_p()
    _check(_fn("chf_pattern_from_csr")(int(nb), rpp, cip, C.byref(out)))
    return Pattern(out)


def pattern_adaptive(A: Bsr, tmax: int, tau: float = 1.0, p0: Pattern | None = None) -> Pattern:
    out = C.c_void_p()
    _check(_fn("chf_pattern_adaptive")(A.h, p0.h if p0 is not None else None, int(tmax), float(tau),
                                       C.byref(out)))
    return Pattern(out)


def pattern_template(nx, ny, nz, offsets) -> Pattern:
    """offsets: int array [noff, 3] of (dx, dy, dz), each to a smaller index."""
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1, 3))
    out = C.c_void_p()
    _check(_fn("chf_pattern_template")(int(nx), int(ny), int(nz), off.shape[0], off.ctypes.data_as(C.c_void_p),
                                       C.byref(out)))
    return Pattern(out)


def pattern_export(P: Pattern):
    nb, nnz = C.c_int64(), C.c_int64()
    _check(_fn("chf_pattern_info")(P.h, C.byref(nb), C.byref(nnz)))
    rowptr = np.empty(nb.value + 1, np.int64)
    colidx = np.empty(nnz.value, np.int32)
    _check(_fn("chf_pattern_export")(P.h, rowptr.ctypes.data_as(C.c_void_p), colidx.ctypes.data_as(C.c_void_p)))
    return rowptr, colidx


# ------------------------------------------------------------------- FSAI --
def fsai_setup(A: Bsr, P: Pattern, g_store=F64) -> Fsai:
    out = C.c_void_p()
    bad = C.c_int64(-1)
    rc = _fn("chf_fsai_setup")(A.h, P.h, g_store, C.byref(out), C.byref(bad))
    if rc != 0:
        err = ChfError(rc, lib().chf_last_error().decode())
        err.bad_row = bad.value
        raise err
    return Fsai(out)


def bsr_triple(A: Bsr, G: Fsai) -> Bsr:
    """G A G^T (the matrix the inner factor of nested FSAI is built for)."""
    out = C.c_void_p()
    _check(_fn("chf_bsr_triple")(A.h, G.h, C.byref(out)))
    return Bsr(out)


def fsai_nest(G0: Fsai, G1: Fsai) -> Fsai:
    """Nested factor M = G0^T G1^T G1 G0; keeps G0 and G1 alive."""
    out = C.c_void_p()
    _check(_fn("chf_fsai_nest")(G0.h, G1.h, C.byref(out)))
    n = Fsai(out)
    n._parts = (G0, G1)
    return n


def fsai_export(G: Fsai, nnz: int, b: int):
    vals = np.empty((nnz, b, b), np.float64)
    _check(_fn("chf_fsai_export")(G.h, vals.ctypes.data_as(C.c_void_p)))
    return vals


def fsai_export_flat(G: Fsai, nvals: int):
    """G's values as one flat array (variable block sizes: nvals values)."""
    vals = np.empty(nvals, np.float64)
    _check(_fn("chf_fsai_export")(G.h, vals.ctypes.data_as(C.c_void_p)))
    return vals


def fsai_apply(G: Fsai, r, z, work, dtype=F64, stream=None):
    _check(_fn("chf_fsai_apply")(G.h, dtype, _ptr(r), _ptr(z), _ptr(work), _stream(stream)))


def lmax_lanczos(A: Bsr, G: Fsai, v0, iters=100, safety=1.01, dtype=F64, stream=None):
    beta, theta = C.c_double(), C.c_double()
    _check(_fn("chf_lmax_lanczos")(A.h, G.h, dtype, int(iters), _ptr(v0), float(safety), C.byref(beta),
                                   C.byref(theta), _stream(stream)))
    return beta.value, theta.value


def cheb4_smooth(A: Bsr, G: Fsai, beta, degree, b, x, x_is_zero=False, work=None, dtype=F64, stream=None):
    _check(_fn("chf_cheb4_smooth")(A.h, G.h, dtype, float(beta), int(degree), _ptr(b), _ptr(x),
                                   int(bool(x_is_zero)), _ptr(work), _stream(stream)))


def cheb4_smooth_noalloc(A: Bsr, G: Fsai, beta, degree, b, x, x_is_zero=False, dtype=F64, stream=None):
    _check(_fn("chf_cheb4_smooth_noalloc")(A.h, G.h, int(dtype), float(beta), int(degree), _ptr(b), _ptr(x),
                                           int(bool(x_is_zero)), _stream(stream)))


def cheb1_smooth(A: Bsr, G: Fsai, alpha, beta, degree, b, x, x_is_zero=False, work=None, dtype=F64, stream=None):
    _check(_fn("chf_cheb1_smooth")(A.h, G.h, dtype, float(alpha), float(beta), int(degree), _ptr(b), _ptr(x),
                                   int(bool(x_is_zero)), _ptr(work), _stream(stream)))


def richardson_smooth(A: Bsr, G: Fsai, omega, degree, b, x, x_is_zero=False, work=None, dtype=F64, stream=None):
    _check(_fn("chf_richardson_smooth")(A.h, G.h, dtype, float(omega), int(degree), _ptr(b), _ptr(x),
                                        int(bool(x_is_zero)), _ptr(work), _stream(stream)))


# ----------------------------------------------------------------- levels --
def levels_create(A0: Bsr) -> Levels:
    out = C.c_void_p()
    _check(_fn("chf_levels_create")(A0.h, C.byref(out)))
    lv = Levels(out)
    lv._a0 = A0      # keep the finest operator alive
    return lv


def levels_add_coarse(L: Levels, nc, p_rowptr, p_colidx, p_vals, basis=None):
    """basis: host float64 (nf, b, b) block-diagonal T of P = T (P_s (x) I_b), or None."""
    rp, rpp = _host(p_rowptr, np.int64)
    ci, cip = _host(p_colidx, np.int32)
    pv, pvp = _host(p_vals, np.float64)
    tb, tbp = (None, None) if basis is None else _host(basis, np.float64)
    _check(_fn("chf_levels_add_coarse")(L.h, int(nc), rpp, cip, pvp, tbp))


def levels_setup(L: Levels, degree=4, pattern=0, tmax=0, tau=1.0, lanczos_iters=100, safety=1.01, dtype=F64,
                 v0=None):
    """pattern: 0 lower(A), 1 adaptive, 2 diagonal. v0: list of device
    float64 tensors (one per level except the coarsest) or None."""
    opts = LevelOpts(int(degree), int(pattern), int(tmax), float(tau), int(lanczos_iters), float(safety),
                     int(dtype))
    arr = None
    if v0 is not None:
        arr = (C.c_void_p * len(v0))(*[C.c_void_p(t.data_ptr()) if t is not None else None for t in v0])
    bad = C.c_int64(-1)
    rc = _fn("chf_levels_setup")(L.h, C.byref(opts), arr, C.byref(bad))
    if rc != 0:
        err = ChfError(rc, lib().chf_last_error().decode())
        err.bad_row = bad.value
        raise err


def levels_set_pattern(L: Levels, level: int, P: Pattern):
    _check(_fn("chf_levels_set_pattern")(L.h, int(level), P.h))


def levels_info(L: Levels):
    nl = C.c_int()
    _check(_fn("chf_levels_info")(L.h, C.byref(nl), None))
    nbs = np.empty(nl.value, np.int64)
    _check(_fn("chf_levels_info")(L.h, C.byref(nl), nbs.ctypes.data_as(C.c_void_p)))
    return nbs


def levels_get(L: Levels, level: int):
    a, g, p = C.c_void_p(), C.c_void_p(), C.c_void_p()
    _check(_fn("chf_levels_get")(L.h, int(level), C.byref(a), C.byref(g), C.byref(p)))
    return (Bsr(a, owner=False), Fsai(g, owner=False) if g.value else None,
            Pattern(p, owner=False) if p.value else None)


def levels_get_beta(L: Levels, level: int) -> float:
    v = C.c_double()
    _check(_fn("chf_levels_get_beta")(L.h, int(level), C.byref(v)))
    return v.value


def levels_set_beta(L: Levels, level: int, beta: float):
    _check(_fn("chf_levels_set_beta")(L.h, int(level), float(beta)))


def levels_set_nesting(L: Levels, nest=1):
    _check(_fn("chf_levels_set_nesting")(L.h, int(nest)))


def levels_set_cycle(L: Levels, smoother=SMOOTH_CHEB4, param=0.0, cycle=CYCLE_VKK):
    _check(_fn("chf_levels_set_cycle")(L.h, int(smoother), float(param), int(cycle)))


def vcycle(L: Levels, b, x, x_is_zero=True, stream=None):
    _check(_fn("chf_vcycle")(L.h, _ptr(b), _ptr(x), int(bool(x_is_zero)), _stream(stream)))


def levels_energy_factor(L: Levels, e0, tol=1e-8, maxit=50, stream=None):
    """Returns (rho_A, cycles) of the hierarchy's cycle from the error e0
    (device double[N], not modified)."""
    rho, cyc = C.c_double(), C.c_int()
    _check(_fn("chf_levels_energy_factor")(L.h, _ptr(e0), float(tol), int(maxit), C.byref(rho), C.byref(cyc),
                                           _stream(stream)))
    return rho.value, cyc.value


def pcg_solve(L: Levels, b, x, rtol=1e-8, maxit=200, flexible=False, stream=None, raise_on_noconv=True):
    """Returns (iterations, relative residual history, true relative residual, status)."""
    iters = C.c_int()
    hist = np.zeros(maxit + 1, np.float64)
    tr = C.c_double()
    rc = _fn("chf_pcg_solve")(L.h, _ptr(b), _ptr(x), float(rtol), int(maxit), int(bool(flexible)),
                              C.byref(iters), hist.ctypes.data_as(C.c_void_p), C.byref(tr), _stream(stream))
    if rc != 0 and not (rc == CHF_ENOCONV and not raise_on_noconv):
        _check(rc)
    return iters.value, hist[:iters.value + 1], tr.value, rc


def bicgstab_solve(L: Levels, b, x, rtol=1e-8, maxit=200, stream=None, raise_on_noconv=True):
    """Returns (iterations, residual history per half step, true relative residual, status)."""
    iters = C.c_int()
    hist = np.full(2 * maxit + 1, np.nan, np.float64)
    tr = C.c_double()
    rc = _fn("chf_bicgstab_solve")(L.h, _ptr(b), _ptr(x), float(rtol), int(maxit), C.byref(iters),
                                   hist.ctypes.data_as(C.c_void_p), C.byref(tr), _stream(stream))
    if rc != 0 and not (rc == CHF_ENOCONV and not raise_on_noconv):
        _check(rc)
    return iters.value, hist[~np.isnan(hist)], tr.value, rc


# -------------------------------------------------------------------- MLP --
def mlp_candidates(A: Bsr):
    n = C.c_int64()
    _check(_fn("chf_mlp_candidates")(A.h, C.byref(n), None, None))
    nb = A.info()[0]
    rowptr = np.empty(nb + 1, np.int64)
    cols = np.empty(n.value, np.int32)
    _check(_fn("chf_mlp_candidates")(A.h, C.byref(n), rowptr.ctypes.data_as(C.c_void_p),
                                     cols.ctypes.data_as(C.c_void_p)))
    return rowptr, cols


def mlp_features(A: Bsr, nx: int, ny: int, feats, stream=None):
    _check(_fn("chf_mlp_features")(A.h, int(nx), int(ny), _ptr(feats), _stream(stream)))


def mlp_create(params) -> Mlp:
    p, pp = _host(params, np.float32)
    out = C.c_void_p()
    _check(_fn("chf_mlp_create")(pp, C.byref(out)))
    return Mlp(out)


def mlp_get_params(net: Mlp):
    out = np.empty(NPARAM, np.float32)
    _check(_fn("chf_mlp_get_params")(net.h, out.ctypes.data_as(C.c_void_p)))
    return out


def mlp_forward(net: Mlp, feats, n: int, logits, stream=None):
    _check(_fn("chf_mlp_forward")(net.h, _ptr(feats), int(n), _ptr(logits), _stream(stream)))


def mlp_loss_grad(net: Mlp, feats, labels, n: int, grad, stream=None):
    loss = C.c_float()
    _check(_fn("chf_mlp_loss_grad")(net.h, _ptr(feats), _ptr(labels), int(n), C.byref(loss), _ptr(grad),
                                    _stream(stream)))
    return loss.value


def mlp_train_step(net: Mlp, feats, labels, n: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    loss = C.c_float()
    _check(_fn("chf_mlp_train_step")(net.h, _ptr(feats), _ptr(labels), int(n), float(lr), float(beta1),
                                     float(beta2), float(eps), C.byref(loss), _stream(stream)))
    return loss.value


def mlp_propose(A: Bsr, net: Mlp, nx: int, ny: int, t: int) -> Pattern:
    out = C.c_void_p()
    _check(_fn("chf_mlp_propose")(A.h, net.h, int(nx), int(ny), int(t), C.byref(out)))
    return Pattern(out)


def mlp_labels(A: Bsr, P: Pattern, labels, stream=None):
    _check(_fn("chf_mlp_labels")(A.h, P.h, _ptr(labels), _stream(stream)))


def mlp_train(net: Mlp, feats, labels, n: int, perm=None, batch=8192, epochs=1, lr=1e-3, beta1=0.9, beta2=0.999,
              eps=1e-8, stream=None):
    """Returns the mean loss of each epoch."""
    hist = np.zeros(max(epochs, 1), np.float32)
    _check(_fn("chf_mlp_train")(net.h, _ptr(feats), _ptr(labels), int(n), _ptr(perm), int(batch), int(epochs),
                                float(lr), float(beta1), float(beta2), float(eps), hist.ctypes.data_as(C.c_void_p),
                                _stream(stream)))
    return hist[:epochs]
