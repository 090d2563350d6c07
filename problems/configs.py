"""The five workloads: sizes, block sizes, hierarchy depth and solver knobs."""
from __future__ import annotations

from dataclasses import dataclass


@dataclass(frozen=True)
class ProblemConfig:
    name: str
    n: int              # finest patches per side
    dim: int
    b: int              # block size C(p+d, d)
    power: int          # D = L^power (2: biharmonic-like, 3: triharmonic-like)
    levels: int         # V-cycle levels, finest included
    pattern: str        # "lower" (static lower(A)) or "adaptive" (Algorithm 1)
    tmax: int           # adaptive steps (max off-diagonal blocks per row)
    degree: int         # Chebyshev degree k (V(k,k))
    precision: str      # "f64", "f32" (A, G FP32) or "bf16g" (A FP32, G BF16)
    rtol: float
    seed: int = 0
    transfer_order: int = 2   # interpolation nodes per direction of the patch transfer (2 bilinear, 4 cubic)


CONFIGS = {
    # 32x32 patches, b = 10 (cubic 2D PUM), static lower(A) pattern, 3 levels.
    "c0": ProblemConfig("c0-biharm2d-32", 32, 2, 10, 2, 3, "lower", 0, 3, "f64", 1e-8),
    # 512x512 patches, b = 10, adaptive t_max = 8, 6 levels, degree 4.
    "c1": ProblemConfig("c1-biharm2d-512", 512, 2, 10, 2, 6, "adaptive", 8, 4, "f64", 1e-8),
    # 256x256 patches, b = 21 (quintic 2D PUM), triharmonic-like, mixed; cubic
    # patch transfer (a sixth-order operator needs transfer orders summing past 6).
    "c2": ProblemConfig("c2-triharm2d-256", 256, 2, 21, 3, 5, "adaptive", 8, 4, "f32", 1e-10, transfer_order=4),
    # 64^3 patches, b = 10 (quadratic 3D PUM), batched setup only.
    "c3": ProblemConfig("c3-biharm3d-64", 64, 3, 10, 2, 1, "adaptive", 23, 4, "f64", 1e-8),
    # learned-pattern test grid: as c1.
    "c4": ProblemConfig("c4-learned-512", 512, 2, 10, 2, 6, "learned", 8, 4, "f64", 1e-8),
}
