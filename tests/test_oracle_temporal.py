"""Pins of the oracle's temporal integration (Section 3.4.1): with alpha =
N_old / (N_old + N_new) the blend is the pooled mean of every sample seen,
and the stored count follows the threshold heuristic."""
import numpy as np

import oracle
import synth

U = 2.0 ** -24


def _run(frames, max_samples):
    """frames: list of (keys ascending, values [G,3], counts [G]); returns the final state."""
    pk = np.zeros(0, np.uint64); pv = np.zeros((0, 3), np.float32); pc = np.zeros(0, np.uint32)
    for k, v, c in frames:
        pv, pc = oracle.temporal_integrate(k, v, c, pk, pv, pc, max_samples)
        pk = k
    return pk, pv, pc


def test_pooled_mean_without_threshold():
    rng = np.random.default_rng(3)
    G, T = 200, 12
    keys = np.arange(G, dtype=np.uint64) * 7 + 1
    vals = [rng.uniform(0.01, 5, (G, 3)).astype(np.float32) for _ in range(T)]
    cnts = [rng.integers(1, 60, G).astype(np.uint32) for _ in range(T)]
    _, v, c = _run(list(zip([keys] * T, vals, cnts)), 1 << 24)
    n = np.sum(cnts, axis=0).astype(np.float64)
    exact = sum(cnts[t][:, None].astype(np.float64) * vals[t] for t in range(T)) / n[:, None]
    assert np.array_equal(c, n.astype(np.uint32))
    # each step rounds alpha, two products and a sum: a few ulps per frame at most
    assert np.all(np.abs(v - exact) <= 4 * T * U * exact)


def test_threshold_keeps_the_history_weight():
    # with N new samples per frame and threshold M, once the count reaches M the
    # blend is a moving average with alpha = M / (M + N); compare with float64
    M, N, T = 50, 7, 30
    keys = np.array([3], np.uint64)
    rng = np.random.default_rng(8)
    xs = [rng.uniform(0.5, 2, (1, 3)).astype(np.float32) for _ in range(T)]
    frames = [(keys, xs[t], np.array([N], np.uint32)) for t in range(T)]
    _, v, c = _run(frames, M)
    assert int(c[0]) == M
    ref, n = xs[0].astype(np.float64), min(N, M)
    for t in range(1, T):
        a = n / (n + N)
        ref = a * ref + (1 - a) * xs[t]
        n = min(n + N, M)
    assert np.all(np.abs(v - ref) <= 8 * T * U * ref)


def test_absent_keys_start_over_and_counts_are_capped():
    k0 = np.array([1, 2], np.uint64); k1 = np.array([2, 9], np.uint64)
    v0 = np.array([[1, 1, 1], [2, 2, 2]], np.float32); v1 = np.array([[4, 4, 4], [5, 5, 5]], np.float32)
    v, c = oracle.temporal_integrate(k1, v1, np.array([3, 99], np.uint32), k0, v0, np.array([1, 1], np.uint32), 10)
    assert np.array_equal(v[1], v1[1]) and int(c[1]) == 10          # new key: its own average, count capped
    assert np.allclose(v[0], (2 * 1 + 4 * 3) / 4, rtol=4 * U) and int(c[0]) == 4


def test_frames_integrate_to_the_pooled_fixed_point_sums():
    """Whole path: the same geometry with fresh noise each frame and a fixed
    jitter seed keeps the cells, so after T frames each cell holds the mean
    of all its samples: sum over frames of the cell sums over the sum of the
    counts (the pinned fixed-point group-by), within T rounding steps."""
    f = synth.generate(synth.get("tiny_64x64"), frame=0)
    truth = f["truth"].numpy()
    rng = np.random.default_rng(11)
    state, S, N = None, None, None
    T = 6
    for t in range(T):
        m = np.exp(rng.normal(size=truth.shape) - 0.5).astype(np.float32)
        noisy = (truth * m).astype(np.float32)
        g = dict(f)
        g["r"], g["g"], g["b"] = noisy[:, 0].copy(), noisy[:, 1].copy(), noisy[:, 2].copy()
        R = oracle.filter_frame(g, prev_state=state, temporal=True, max_samples=1 << 24)
        assert R.table.order_free
        S = R.gsum.astype(np.float64) * 2.0 ** -24 if S is None else S + R.gsum * 2.0 ** -24
        N = R.gcnt.astype(np.float64) if N is None else N + R.gcnt
        state = R.state
    pooled = S / N[:, None]
    k, v, c = state
    assert np.array_equal(k, R.gkey) and np.array_equal(c, N.astype(np.uint32))
    assert np.all(np.abs(v - pooled) <= (4 * T + 1) * U * np.abs(pooled) + 1e-7)
