"""Seeded per-vertex throughput for the pixel resolve.

The generator gives each vertex its contribution directly; the attenuation
from the camera to a vertex is not modelled, so the resolve is exercised with
a synthetic RGB throughput, uniform in [0, 1) per vertex and channel.

This module only makes inputs; it holds none of the filter's arithmetic.
"""
from __future__ import annotations

import torch

from .rng import derive_key, rand_uniform


def synthetic_throughput(n: int, seed: int = 1902, device="cpu"):
    idx = torch.arange(n, dtype=torch.int64, device=device)
    return tuple(rand_uniform(derive_key(seed, 0x7468 + c), idx) for c in range(3))
