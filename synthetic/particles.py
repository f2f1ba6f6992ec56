"""Seeded particle positions: uniform on [0, 2*pi)^3, FP64, layout X[Np][3]."""
from __future__ import annotations

import math


def uniform_particles(Np: int, seed: int, device="cpu"):
    """torch float64 tensor [Np, 3] of uniform positions (x1, x2, x3)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    X = torch.rand((Np, 3), generator=gen, device=device, dtype=torch.float64)
    X *= 2.0 * math.pi
    return X
