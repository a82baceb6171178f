"""Counter-based random numbers for the synthetic scene generator.

The generator draws every random number from a stateless hash of
(key, element index), so a frame is reproducible on any device and in any
order.  The 32-bit mixer is the "PCG hash" of Jarzynski and Olano,
"Hash Functions for GPU Rendering", JCGT 9(3), 2020 (an LCG step followed by
the PCG RXS-M-XS output permutation).  Tensors hold uint32 values in int64
so that every product stays below 2^63.

This module only makes inputs; it holds none of the filter's arithmetic.
"""
from __future__ import annotations

import torch

M32 = 0xFFFFFFFF
M64 = 0xFFFFFFFFFFFFFFFF


def splitmix64(x: int) -> int:
    """SplitMix64 output function on a Python int (Steele, Lea, Flood 2014)."""
    z = (x + 0x9E3779B97F4A7C15) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def derive_key(*parts: int) -> int:
    """Fold integers (seed, frame, purpose, ...) into one 64-bit key."""
    k = 0
    for p in parts:
        k = splitmix64(k ^ (p & M64))
    return k


def pcg_hash(x: torch.Tensor) -> torch.Tensor:
    """PCG hash of uint32 values held in an int64 tensor."""
    state = (x * 747796405 + 2891336453) & M32
    word = (((state >> ((state >> 28) + 4)) ^ state) * 277803737) & M32
    return ((word >> 22) ^ word) & M32


def rand_u32(key: int, idx: torch.Tensor) -> torch.Tensor:
    """uint32 (in int64) for each element index under a 64-bit key."""
    lo = key & M32
    hi = (key >> 32) & M32
    return pcg_hash((pcg_hash((idx & M32) ^ lo) + hi) & M32)


def rand_uniform(key: int, idx: torch.Tensor) -> torch.Tensor:
    """float32 uniform in [0, 1) with 24 random bits."""
    return (rand_u32(key, idx) >> 8).to(torch.float32) * (1.0 / 16777216.0)


def rand_normal(key: int, idx: torch.Tensor) -> torch.Tensor:
    """float32 standard normal by the Box-Muller transform."""
    u1 = 1.0 - rand_uniform(derive_key(key, 1), idx)  # (0, 1]
    u2 = rand_uniform(derive_key(key, 2), idx)
    return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * torch.pi * u2)


class HostRng:
    """Scalar stream for scene layout (box sizes, albedos) on the host."""

    def __init__(self, key: int):
        self.key = key
        self.ctr = 0

    def uniform(self) -> float:
        self.ctr += 1
        return (splitmix64(self.key ^ (self.ctr * 0xD1B54A32D192ED03 & M64)) >> 40) / float(1 << 24)
