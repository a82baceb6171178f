"""Pins of the oracle's pixel resolve (Section 3: each selected vertex's
value times its throughput, accumulated in its pixel): exact sums of small
integers against Python integers, a missing throughput as a throughput of
one, masked vertices contributing nothing, accumulation onto a given image,
and the stated order of the binary32 sums (bounce 0 first)."""
import numpy as np

import oracle


def _layout(P, V, rng, lo=-50, hi=50):
    c = rng.integers(lo, hi, (P * V, 3)).astype(np.float32)
    t = rng.integers(0, 8, (P * V, 3)).astype(np.float32)
    return c, t


def test_exact_integer_sums_match_python_integers():
    rng = np.random.default_rng(1)
    for P, V in ((1, 1), (7, 3), (1000, 4)):
        c, t = _layout(P, V, rng)
        valid = (rng.random(P * V) < 0.8).astype(np.uint8)
        got = oracle.resolve_pixels(c, t, valid, P, V)
        for p in range(0, P, max(1, P // 50)):
            for ch in range(3):
                exp = sum(int(t[b * P + p, ch]) * int(c[b * P + p, ch]) for b in range(V) if valid[b * P + p])
                assert got[p, ch] == exp


def test_missing_throughput_is_one_and_masked_vertices_add_nothing():
    rng = np.random.default_rng(2)
    P, V = 300, 3
    c, _ = _layout(P, V, rng)
    valid = (rng.random(P * V) < 0.7).astype(np.uint8)
    a = oracle.resolve_pixels(c, None, valid, P, V)
    b = oracle.resolve_pixels(c, np.ones_like(c), valid, P, V)
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    c2 = c.copy()
    c2[valid == 0] = np.nan
    assert np.array_equal(oracle.resolve_pixels(c2, None, valid, P, V).view(np.uint32), a.view(np.uint32))


def test_accumulates_onto_a_given_image():
    rng = np.random.default_rng(3)
    P, V = 200, 2
    c, t = _layout(P, V, rng)
    init = rng.integers(-100, 100, (P, 3)).astype(np.float32)
    got = oracle.resolve_pixels(c, t, None, P, V, init=init)
    assert np.array_equal(got, init + oracle.resolve_pixels(c, t, None, P, V))


def test_sums_run_from_the_first_bounce():
    # (1e8 + 1) - 1e8 is 0 in binary32, other orders give 1
    c = np.array([[1e8] * 3, [1.0] * 3, [-1e8] * 3], np.float32)
    got = oracle.resolve_pixels(c, None, None, 1, 3)
    assert np.all(got == 0.0)
