"""Seeded initial weights of the sparse-cell MLP (an input, like the vertex
streams: both the GPU path and the reference start from these values).

Packed float32 layout: W1 [64, 80], b1 [64], W2 [64, 64], b2 [64],
W3 [16, 64] (rows 3..15 zero), b3 [16] (zero).  He-uniform weights
(bound sqrt(6 / fan_in)), zero biases.
"""
from __future__ import annotations

import numpy as np

SHAPES = [(64, 80), (64,), (64, 64), (64,), (16, 64), (16,)]
N_PARAM = sum(int(np.prod(s)) for s in SHAPES)


def init_params(seed: int = 1902) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    for shp in SHAPES:
        if len(shp) == 2:
            bound = np.sqrt(6.0 / shp[1])
            w = rng.uniform(-bound, bound, shp)
            if shp[0] == 16:
                w[3:] = 0.0
        else:
            w = np.zeros(shp)
        parts.append(w.astype(np.float32).reshape(-1))
    return np.concatenate(parts)
