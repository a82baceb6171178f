"""A seeded point cloud with normals in every direction.

The scenes' surfaces are axis-aligned, so almost every voxel holds one
normal class; the search for similar normals along a probe run needs voxels
that share a position under several classes.  This cloud puts n vertices
uniformly in a cube of half-width `spread` centred at (0, 1, 0), with
normals drawn isotropically and about 15% of their components set to zero
(renormalised), and contributions uniform in [0.05, 2).  Every vertex is
valid.  The camera, scale and table parameters of the returned frame match
what the filter takes.

This module only makes inputs; it holds none of the filter's arithmetic.
"""
from __future__ import annotations

import numpy as np


def mixed_normals_frame(n: int, seed: int, s: float, spread: float = 0.6, log2_slots: int = 15):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(-spread, spread, (n, 3)).astype(np.float32)
    pos[:, 1] += 1.0
    nrm = rng.normal(size=(n, 3))
    nrm[rng.random((n, 3)) < 0.15] = 0.0
    nrm[np.all(nrm == 0, 1), 0] = 1.0
    nrm = (nrm / np.linalg.norm(nrm, axis=1, keepdims=True)).astype(np.float32)
    rgb = rng.uniform(0.05, 2.0, (n, 3)).astype(np.float32)
    return {"px": pos[:, 0], "py": pos[:, 1], "pz": pos[:, 2], "nx": nrm[:, 0], "ny": nrm[:, 1], "nz": nrm[:, 2],
            "r": rgb[:, 0], "g": rgb[:, 1], "b": rgb[:, 2], "valid": np.ones(n, np.uint8),
            "cam": (0.0, 2.0, -6.0), "s": s, "seed": 7, "log2_slots": log2_slots, "max_probe": 64, "frac_bits": 24}
