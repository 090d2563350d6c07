"""The C-ABI library loads and exports every entry point that include/chf.h
declares (no GPU needed: nothing is computed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "chf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(chf_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["chf_bsr_create", "chf_fsai_setup", "chf_cheb4_smooth", "chf_vcycle", "chf_pcg_solve",
                 "chf_pattern_adaptive", "chf_lmax_lanczos", "chf_mlp_train_step"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2509_06744_amd import binding
    if not os.path.exists(binding.lib_path):
        pytest.fail("libchf.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(binding.lib_path)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, f"not exported: {missing}"
    # every declared entry point has a binding with the same name
    assert set(declared()) <= set(binding.EXPORTED)


def test_version_string():
    import paper_2509_06744_amd as chf
    assert "gfx950" in chf.version()


def test_binding_exports_every_wrapper():
    # every public wrapper defined in the binding is re-exported by the package
    import inspect

    from paper_2509_06744_amd import binding
    defined = {n for n, f in vars(binding).items()
               if inspect.isfunction(f) and not n.startswith("_") and f.__module__ == binding.__name__}
    assert defined <= set(binding.__all__), sorted(defined - set(binding.__all__))
