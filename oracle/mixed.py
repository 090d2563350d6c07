"""Rounded operators for the mixed-precision form (storage of A and G in
FP32 or BF16, round to nearest even). BF16 values are obtained by rounding
to FP32 first and then to BF16, the same two steps the storage conversion
takes. Parity of the mixed form is unpinned beyond these roundings: its error
against the FP64 oracle is reported, not derived."""
from __future__ import annotations

import numpy as np


def round_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_bf16(x):
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
