"""Synthetic key streams for table-load sweeps.

A real scene at 3840x2160x4 fills a 2^25-slot table to a few percent at the
default scale, and never above its valid-vertex count; the insert and the
lookup only see keys, so loads up to 0.7 are reached by handing them keys
drawn from `distinct` cell ids.  Vertex i < distinct takes id i (so exactly
`distinct` cells exist), later vertices a uniformly random id.  The key of
id c is c * 2654435761 (odd, so distinct ids give distinct keys; below 2^57,
so the reserved top bits stay 0).  Contributions are uniform in [0, 1).

This module only makes inputs; it holds none of the filter's arithmetic.
"""
from __future__ import annotations

import torch

from .rng import derive_key, rand_u32, rand_uniform


def synthetic_keys(n: int, distinct: int, seed: int = 1902, device="cpu"):
    assert 0 < distinct <= n and distinct < (1 << 30)
    idx = torch.arange(n, dtype=torch.int64, device=device)
    pick = (rand_u32(derive_key(seed, 0x6B657973), idx) * distinct) >> 32
    cid = torch.where(idx < distinct, idx, pick)
    key = cid * 2654435761
    r = rand_uniform(derive_key(seed, 1), idx)
    g = rand_uniform(derive_key(seed, 2), idx)
    b = rand_uniform(derive_key(seed, 3), idx)
    return {"key": key, "r": r, "g": g, "b": b, "valid": torch.ones(n, dtype=torch.uint8, device=device)}
