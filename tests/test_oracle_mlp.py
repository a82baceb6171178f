"""Pins of the MLP reference: bfloat16 rounding closed forms, exact values of
the positional encoding, a forward pass with a closed-form result, the
backward pass against float64 finite differences, and Adam's closed-form
first step and convergence on a convex problem."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from synth.mlp_init import init_params


def test_bf16_rounding_closed_forms():
    f = np.float32
    cases = {1.0: 1.0, 1 + 2.0 ** -8: 1.0, 1 + 3 * 2.0 ** -8: 1 + 2.0 ** -6, 1 + 2.0 ** -7: 1 + 2.0 ** -7,
             1 + 2.0 ** -8 + 2.0 ** -20: 1 + 2.0 ** -7, -2.5: -2.5, 0.0: 0.0, 3.0e38: 3.0040553e38, 3.4e38: np.inf}
    for x, want in cases.items():
        assert mlp.bf16_round(np.array([x], f))[0] == f(want), x
    neg0 = mlp.bf16_round(np.array([-0.0], f))[0]
    assert neg0 == 0 and np.signbit(neg0)
    assert np.isnan(mlp.bf16_round(np.array([np.nan], f))[0])
    assert mlp.bf16_round(np.array([np.inf], f))[0] == np.inf
    r = np.random.default_rng(0).normal(size=10000).astype(f)
    b = mlp.bf16_round(r)
    assert np.all((b.view(np.uint32) & 0xFFFF) == 0)
    assert np.all(np.abs(b - r) <= np.abs(r) * 2.0 ** -8)


def _keys_for(q, lp, code=4):
    q = np.asarray(q, np.int64)
    return ((q[:, 0] + 65536) | ((q[:, 1] + 65536) << 17) | ((q[:, 2] + 65536) << 34) |
            ((np.asarray(lp) + 16) << 51) | (code << 56)).astype(np.uint64)


def test_key_decoding_matches_the_oracle_key_layout():
    """Cell-centre vertices (closed form x~ = k) decode back to k and l'."""
    rng = np.random.default_rng(2)
    n = 500
    h = np.float32(0.01) * np.float32(64)
    kx, kz = rng.integers(-20, 20, n), rng.integers(-20, 20, n)
    pos = np.stack([(kx + 0.5) * h, np.zeros(n), (kz + 0.5) * h], 1).astype(np.float32)
    nrm = np.tile(np.array([[0, 1, 0]], np.float32), (n, 1))
    k = oracle.build_keys(pos[:, 0], pos[:, 1], pos[:, 2], nrm[:, 0], nrm[:, 1], nrm[:, 2], None,
                          (0.0, 0.0, -100.0), 0.01, 3, 0, 14)
    q, lp = mlp.decode_key(k["key"])
    assert np.array_equal(q[:, 0], kx) and np.array_equal(q[:, 2], kz) and np.all(q[:, 1] == 0) and np.all(lp == 6)


def test_positional_encoding_exact_values():
    # p = (q + 1/2) 2^(l' - 10); choose l' = 9 so p = (q + 1/2) / 2
    q = np.array([[0, -1, 1], [2, 5, -4]], np.int64)
    lp = np.array([9, 9])
    x = mlp.features(_keys_for(q, lp), np.array([[1, 2, 3], [0, 0, 1]], np.float32),
                     np.array([[0, 1, 0], [0.6, 0, 0.8]], np.float32), (0.0, 0.0, 0.0))
    p = (q + 0.5) / 2.0
    for k in range(12):
        t = p * 2.0 ** k
        s, c = x[:, 6 * k: 6 * k + 3], x[:, 6 * k + 3: 6 * k + 6]
        for val, ref in ((s, np.sin(np.pi * t)), (c, np.cos(np.pi * t))):
            assert np.all(np.abs(val - ref) <= np.abs(ref) * 2.0 ** -8 + 1e-9)   # ref is unreduced
    # k = 2: 4p = 2q + 1 is odd -> sin exactly 0, cos exactly -1; k >= 3: 2^k p is even -> 0 and 1
    assert np.all(x[:, 12:15] == 0) and np.all(x[:, 15:18] == -1)
    for k in range(3, 12):
        assert np.all(x[:, 6 * k: 6 * k + 3] == 0) and np.all(x[:, 6 * k + 3: 6 * k + 6] == 1)
    assert np.array_equal(x[:, 72:75], mlp.bf16_round(np.array([[0, 1, 0], [0.6, 0, 0.8]], np.float32)))
    v = x[:, 75:78].astype(np.float64)
    assert np.allclose(v[0], np.array([1, 2, 3]) / np.sqrt(14), rtol=2 ** -8)
    assert np.all(x[:, 78:] == 0)


def test_sinpi_cospi_exact_points_and_accuracy():
    t = np.array([0.0, 0.5, 1.0, 1.5, 2.0, -0.5, -1.0, 7.0, 2.0 ** 40 + 0.5, -3.5, 0.25])
    assert list(mlp.sinpi(t)[:10]) == [0, 1, 0, -1, 0, -1, 0, 0, 1, 1]
    assert list(mlp.cospi(t)[:8]) == [1, 0, -1, 0, 1, 0, -1, -1]
    assert abs(mlp.sinpi(0.25) - np.sqrt(0.5)) < 2e-16
    r = np.random.default_rng(1).uniform(-3, 3, 10000)
    r = np.round(r * 2 ** 20) / 2 ** 20
    assert np.max(np.abs(mlp.sinpi(r) - np.sin(np.pi * r))) < 1e-14
    assert np.max(np.abs(mlp.sinpi(r) ** 2 + mlp.cospi(r) ** 2 - 1)) < 1e-15


def test_positional_encoding_is_periodic_in_the_cell_index():
    """Frequency k has period 2^(11-k) cells at level 10 + 0: shifting the
    cell index by 2^12 leaves every feature unchanged."""
    rng = np.random.default_rng(3)
    q = rng.integers(-20000, 20000, (300, 3))
    lp = np.full(300, 0)
    base = mlp.features(_keys_for(q, lp), np.ones((300, 3), np.float32), np.ones((300, 3), np.float32), (0, 0, 0))
    shifted = mlp.features(_keys_for(q + 2 ** 12, lp), np.ones((300, 3), np.float32), np.ones((300, 3), np.float32),
                           (0, 0, 0))
    assert np.array_equal(base[:, :72], shifted[:, :72])


def test_forward_closed_form_identity_network():
    """W1 copies feature j to unit j, W2 is the identity, W3 picks units 0..2:
    for non-negative bfloat16 inputs y equals x[:, :3] exactly."""
    th = np.zeros(mlp.N_PARAM)
    P = mlp.unpack(th)
    P["W1"][:, :] = 0; P["W1"][np.arange(64), np.arange(64)] = 1.0
    P["W2"][:, :] = np.eye(64)
    P["W3"][:3, :3] = np.eye(3)
    th = mlp.pack(P)
    x = mlp.bf16_round(np.random.default_rng(4).uniform(0, 3, (50, 80)).astype(np.float32))
    y, _ = mlp.forward(th, x)
    assert np.array_equal(y, x[:, :3].astype(np.float64))
    P["b3"][:3] = [1.0, -2.0, 0.5]
    y2, _ = mlp.forward(mlp.pack(P), x)
    assert np.allclose(y2 - y, [[1.0, -2.0, 0.5]])


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(5)
    th = init_params(7).astype(np.float64)
    th += rng.normal(0, 0.05, th.shape) * (mlp.pack({k: np.ones(s) for k, s in mlp.PARAM_SHAPES}) != 0)
    P = mlp.unpack(th); P["W3"][3:] = 0; P["b3"][3:] = 0; th = mlp.pack(P)
    x = rng.normal(size=(37, 80))
    t = rng.normal(size=(37, 3))
    loss, g = mlp.loss_and_grad(th, x, t, bf16=False)
    live = np.nonzero(mlp.pack({k: (np.ones(s) if k != "W3" and k != "b3" else
                                    np.concatenate([np.ones((3,) + s[1:]), np.zeros((13,) + s[1:])]))
                                for k, s in mlp.PARAM_SHAPES}))[0]
    idx = rng.choice(live, 80, replace=False)
    eps = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += eps; tm[i] -= eps
        fd = (mlp.loss_and_grad(tp, x, t, bf16=False)[0] - mlp.loss_and_grad(tm, x, t, bf16=False)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_padded_outputs_get_no_gradient():
    th = init_params(1).astype(np.float64)
    x = mlp.bf16_round(np.random.default_rng(6).normal(size=(20, 80)).astype(np.float32))
    _, g = mlp.loss_and_grad(th, x, np.ones((20, 3)))
    G = mlp.unpack(g)
    assert np.all(G["W3"][3:] == 0) and np.all(G["b3"][3:] == 0) and np.abs(G["W3"][:3]).sum() > 0


def test_adam_first_step_is_a_signed_learning_rate():
    """After one step m_hat = g and v_hat = g^2, so w moves by lr g/(|g| + eps)."""
    g = np.array([1e-3, -2.0, 5e-5, 0.0, 3.0])
    w, m, v = mlp.adam_step(np.ones(5, np.float32), np.zeros(5), np.zeros(5), g, 1, 1e-3)
    assert np.allclose(w, 1 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-7)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_converges_on_a_convex_least_squares_problem():
    rng = np.random.default_rng(8)
    A = rng.normal(size=(40, 5)); b = rng.normal(size=40)
    w = np.zeros(5, np.float32); m = np.zeros(5); v = np.zeros(5)
    for step in range(1, 3001):
        g = 2 * A.T @ (A @ w.astype(np.float64) - b) / 40
        w, m, v = mlp.adam_step(w, m, v, g, step, 1e-2)
    assert np.allclose(w, np.linalg.lstsq(A, b, rcond=None)[0], atol=1e-3)


def test_init_params_layout():
    th = init_params(1902)
    P = mlp.unpack(th.astype(np.float64))
    assert th.dtype == np.float32 and th.size == mlp.N_PARAM
    assert np.all(P["W3"][3:] == 0) and np.all(P["b1"] == 0)
    assert abs(P["W1"]).max() <= np.sqrt(6 / 80) and abs(P["W2"]).max() <= np.sqrt(6 / 64)
