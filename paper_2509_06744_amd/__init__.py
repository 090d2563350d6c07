"""MI355X (gfx950) library for fourth-kind Chebyshev smoothing with
block-FSAI preconditioners in a Galerkin V-cycle, behind a C ABI.

This module is a thin ctypes binding of ``libchf.so`` (declared in
``include/chf.h``): every function marshals arguments and calls the C entry
point of the same name; all arithmetic of the path runs in the library's HIP
kernels. Device vectors are torch tensors on the current HIP device; host
arrays are NumPy arrays. There is no CPU fallback: if the library is missing
the import of the first entry point raises.
"""
from .binding import *  # noqa: F401,F403
from .binding import __all__  # noqa: F401
