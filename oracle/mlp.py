"""MLP reference for the learned sparse-cell fallback -- TEST INFRASTRUCTURE ONLY.

Plain numpy, float64 accumulation.  It states what the GPU's BF16 network
computes so the GPU can be checked against it; only tests/, the smoke check
and the benchmark's CPU-baseline leg may use it.  It shares no code with the
GPU library.

The network (not part of the paper; it stands where Section 3.3 places its
fallbacks for voxels with few vertices):
  features x [80]: positional encoding of the cell centre (12 frequencies,
    sin and cos, 3 axes: 72), the vertex normal (3), the unit view direction
    from the camera (3), two zeros;
  z1 = W1 x + b1, a1 = relu(z1); z2 = W2 a1 + b2, a2 = relu(z2); y = W3 a2 + b3
  with W1 [64, 80], W2 [64, 64], W3 [16, 64] (rows 3..15 unused, kept zero).
BF16 (round to nearest even) is applied to x, to the weights used by the
products (a BF16 copy of the FP32 master weights), to a1 and a2, and to the
back-propagated gradients that enter products (gy, gz2, gz1).  Biases, the
loss and all accumulations are exact (float64 here).  Loss = mean over the
batch and 3 channels of (y - t)^2.  Adam (beta1 0.9, beta2 0.999, eps 1e-8)
updates the float32 master weights.

Positional encoding: with the key's cell index x~ and level l', the centre in
units of s is (x~ + 1/2) 2^l'; p = (x~ + 1/2) 2^(l' - 10) is exact in binary32;
features are sin(pi 2^k p) and cos(pi 2^k p) for k = 0..11 (feature
6k + c is the sine of axis c, 6k + 3 + c its cosine), evaluated in float64
after exact argument reduction (exact at integer and half-integer phases),
and rounded float64 -> float32 -> bfloat16, zeros taken as +0.  The view
direction is
(x - cam) / |x - cam| in float64, rounded the same way.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H, N_OUT_PAD, N_OUT = 80, 64, 16, 3
N_FREQ = 12
PARAM_SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
                ("W3", (N_OUT_PAD, N_H)), ("b3", (N_OUT_PAD,))]
N_PARAM = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


# ------------------------------------------------------------------ bfloat16
def bf16_round(x) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even, NaN kept),
    returned as float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).copy()
    nan = np.isnan(a)
    out[nan] = a[nan]
    return out


def bf16_bits(x) -> np.ndarray:
    return (bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)


def to_bf16_via_f32(x64) -> np.ndarray:
    """float64 -> float32 (nearest) -> bfloat16 (nearest even), as float32."""
    return bf16_round(np.asarray(x64, dtype=np.float64).astype(np.float32))


# ------------------------------------------------------------------ features
def sinpi(t):
    """sin(pi t) for dyadic float64 t: exact reduction to r in [-1/2, 1/2]
    (periodicity 2 and sin(pi t) = sin(pi (1 - t))), then sin(pi r); exact at
    integers and half-integers."""
    r = np.fmod(np.asarray(t, np.float64), 2.0)          # (-2, 2), exact
    r = np.where(r >= 1.0, r - 2.0, r)
    r = np.where(r < -1.0, r + 2.0, r)                    # [-1, 1), exact
    r = np.where(r > 0.5, 1.0 - r, r)
    r = np.where(r < -0.5, -1.0 - r, r)                   # [-1/2, 1/2], exact
    return np.sin(np.pi * r)


def cospi(t):
    return sinpi(np.asarray(t, np.float64) + 0.5)       # exact shift for dyadic t


def decode_key(key):
    k = np.asarray(key, dtype=np.uint64)
    q = np.stack([((k >> np.uint64(17 * c)) & np.uint64(0x1FFFF)).astype(np.int64) - 65536 for c in range(3)], 1)
    lp = ((k >> np.uint64(51)) & np.uint64(31)).astype(np.int64) - 16
    return q, lp


def features(key, pos, nrm, cam) -> np.ndarray:
    """[n, 80] float32 holding bfloat16 values."""
    q, lp = decode_key(key)
    p = (q.astype(np.float64) + 0.5) * np.exp2(lp.astype(np.float64) - 10.0)[:, None]   # exact
    n = p.shape[0]
    x = np.zeros((n, N_IN), np.float64)
    for k in range(N_FREQ):
        t = p * (2.0 ** k)                       # exact dyadic scaling
        x[:, 6 * k: 6 * k + 3] = sinpi(t)
        x[:, 6 * k + 3: 6 * k + 6] = cospi(t)
    x[:, 72:75] = np.asarray(nrm, np.float32).astype(np.float64)
    d = np.asarray(pos, np.float32).astype(np.float64) - np.asarray(cam, np.float32).astype(np.float64)[None, :]
    ss = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
    x[:, 75:78] = d / np.sqrt(ss)[:, None]
    return to_bf16_via_f32(x + 0.0)              # zeros are +0 (IEEE: -0 + 0 = +0)


# ------------------------------------------------------------------ parameters
def unpack(theta):
    out, o = {}, 0
    for name, shp in PARAM_SHAPES:
        sz = int(np.prod(shp))
        out[name] = theta[o:o + sz].reshape(shp)
        o += sz
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).reshape(-1) for name, _ in PARAM_SHAPES])


def forward(theta, x, bf16=True):
    """Returns y [n, 3] and the cache for backward; float64 arithmetic."""
    P = unpack(np.asarray(theta, np.float64))
    rw = (lambda w: bf16_round(w).astype(np.float64)) if bf16 else (lambda w: np.asarray(w, np.float64))
    ra = (lambda a: bf16_round(a.astype(np.float32)).astype(np.float64)) if bf16 else (lambda a: a)
    W1, W2, W3 = rw(P["W1"]), rw(P["W2"]), rw(P["W3"])
    x = np.asarray(x, np.float64)
    z1 = x @ W1.T + P["b1"]
    a1 = ra(np.maximum(z1, 0.0))
    z2 = a1 @ W2.T + P["b2"]
    a2 = ra(np.maximum(z2, 0.0))
    y = a2 @ W3.T + P["b3"]
    cache = (x, z1, a1, z2, a2, W1, W2, W3)
    return y[:, :N_OUT], cache


def loss_and_grad(theta, x, target, bf16=True):
    """MSE loss over batch and channels, and its gradient (packed like theta)."""
    y, (x, z1, a1, z2, a2, W1, W2, W3) = forward(theta, x, bf16)
    B = x.shape[0]
    t = np.asarray(target, np.float64)
    diff = y - t
    loss = float((diff * diff).mean())
    gy = np.zeros((B, N_OUT_PAD))
    gy[:, :N_OUT] = 2.0 * diff / (B * N_OUT)
    rg = (lambda g: bf16_round(g.astype(np.float32)).astype(np.float64)) if bf16 else (lambda g: g)
    gyb = rg(gy)
    g = {"W3": gyb.T @ a2, "b3": gy.sum(0)}
    gz2 = (gyb @ W3) * (z2 > 0)
    gz2b = rg(gz2)
    g["W2"] = gz2b.T @ a1
    g["b2"] = gz2.sum(0)
    gz1 = (gz2b @ W2) * (z1 > 0)
    gz1b = rg(gz1)
    g["W1"] = gz1b.T @ x
    g["b1"] = gz1.sum(0)
    g["W3"][N_OUT:] = 0.0
    g["b3"][N_OUT:] = 0.0
    return loss, pack(g)


def adam_step(w, m, v, grad, step, lr):
    """One Adam update of float32 master weights (step counts from 1)."""
    g = np.asarray(grad, np.float64)
    m = ADAM_B1 * np.asarray(m, np.float64) + (1 - ADAM_B1) * g
    v = ADAM_B2 * np.asarray(v, np.float64) + (1 - ADAM_B2) * g * g
    mh = m / (1 - ADAM_B1 ** step)
    vh = v / (1 - ADAM_B2 ** step)
    w = np.asarray(w, np.float64) - lr * mh / (np.sqrt(vh) + ADAM_EPS)
    return w.astype(np.float32), m.astype(np.float32), v.astype(np.float32)


def predict(theta, x):
    """Inference output: max(0, y)."""
    y, _ = forward(theta, x, bf16=True)
    return np.maximum(y, 0.0)
