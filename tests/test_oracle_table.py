"""Pins of the oracle's accumulation, table simulation, lookup and temporal
blend against facts fixed outside it: conservation of counts and sums,
brute-force group sums, the insertion-order independence and expected probe
lengths of linear probing (Knuth), forced overflow and fingerprint-alias
fixtures, the two limits of the voxel size, exact rational group means, and
the closed form of the exponential moving average."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def _frame_arrays(n, rng, spread=2.0, sigma=1.0):
    pos = rng.uniform(-spread, spread, (n, 3)).astype(np.float32)
    pos[:, 1] = np.abs(pos[:, 1])
    nrm = np.zeros((n, 3), np.float32)
    nrm[np.arange(n), rng.integers(0, 3, n)] = rng.choice([-1.0, 1.0], n)
    rgb = (rng.uniform(0.1, 1.0, (n, 3)) * np.exp(sigma * rng.normal(size=(n, 1)) - sigma * sigma / 2)).astype(np.float32)
    return {"px": pos[:, 0], "py": pos[:, 1], "pz": pos[:, 2], "nx": nrm[:, 0], "ny": nrm[:, 1], "nz": nrm[:, 2],
            "r": rgb[:, 0], "g": rgb[:, 1], "b": rgb[:, 2], "valid": np.ones(n, np.uint8),
            "cam": (0.0, 2.0, -6.0), "s": 0.05, "seed": 99, "log2_slots": 14, "max_probe": 64, "frac_bits": 24}


# ------------------------------------------------------------ group-by
def test_counts_and_sums_are_conserved():
    f = synth.generate(synth.get("tiny_64x64"))
    R = oracle.filter_frame(f, temporal=False)
    ok = R.flags == 0
    assert R.gcnt.sum() == ok.sum()
    assert np.array_equal(R.gsum.sum(0), R.q[ok].sum(0))
    assert np.all(np.diff(R.gkey.astype(np.uint64)) > 0)


def test_group_sums_match_brute_force_dictionary():
    rng = np.random.default_rng(1)
    f = _frame_arrays(3000, rng)
    R = oracle.filter_frame(f, temporal=False)
    d = {}
    for i in np.nonzero(R.flags == 0)[0]:
        c, s = d.get(int(R.key[i]), (0, np.zeros(3, np.int64)))
        d[int(R.key[i])] = (c + 1, s + R.q[i])
    assert len(d) == len(R.gkey)
    for g, K in enumerate(R.gkey):
        c, s = d[int(K)]
        assert c == R.gcnt[g] and np.array_equal(s, R.gsum[g])


def test_fixed_point_rounds_half_to_even():
    r = np.array([0.5, 1.5, 2.5, -0.5, 3.0, 1e30, np.nan, 2**37], np.float32) * np.float32(2.0 ** -24)
    r = np.array(r, np.float32)
    flags = np.zeros(r.shape[0], np.uint8)
    q = oracle.quantize_radiance(r, r, r, 24, flags)
    assert list(q[:5, 0]) == [0, 2, 2, 0, 3]
    assert list(flags) == [0, 0, 0, 0, 0, oracle.RADRANGE, oracle.INVALID, 0]
    flags = np.zeros(1, np.uint8)
    oracle.quantize_radiance(np.array([2.0 ** 40], np.float32), np.zeros(1, np.float32),
                             np.zeros(1, np.float32), 24, flags)
    assert flags[0] == oracle.RADRANGE          # 2^40 * 2^24 >= 2^62


def test_averages_are_exact_group_means_within_half_ulp():
    rng = np.random.default_rng(2)
    f = _frame_arrays(4000, rng)
    f["s"] = 0.5
    R = oracle.filter_frame(f, temporal=False)
    assert R.table.order_free
    for g in range(0, len(R.gkey), 7):
        for c in range(3):
            exact = Fraction(int(R.gsum[g, c]), int(R.gcnt[g]) << 24)
            got = Fraction(float(R.gavg[g, c]))
            ulp = Fraction(float(np.spacing(np.float32(R.gavg[g, c]))))
            assert abs(got - exact) <= ulp / 2 * Fraction(1000001, 1000000)


# ------------------------------------------------------------ limits of the voxel size
def test_tiny_voxels_return_each_vertex_unchanged():
    rng = np.random.default_rng(3)
    f = _frame_arrays(5000, rng)
    f["s"] = 1e-6
    R = oracle.filter_frame(f, temporal=False)
    ok = R.flags == 0
    assert np.all(R.cnt[ok] == 1)
    rgb = np.stack([f["r"], f["g"], f["b"]], 1)
    assert np.abs(R.out[ok] - rgb[ok]).max() <= 2.0 ** -25 + 1e-7


def test_huge_voxel_returns_global_mean():
    """All vertices at the centre of one huge voxel (s = 1 at level 15 gives
    h = 32768; the tangent jitter spans [-h/2, h/2)), so every jittered point
    stays inside it and the lookup returns the global mean."""
    rng = np.random.default_rng(4)
    n = 3000
    f = _frame_arrays(n, rng)
    f["px"] = np.full(n, 16384.0, np.float32); f["pz"] = np.full(n, 16384.0, np.float32)
    f["py"] = rng.uniform(1, 2, n).astype(np.float32)
    f["nx"][:] = 0; f["ny"][:] = 1; f["nz"][:] = 0
    f["cam"] = (16384.0, 1.0e6, 16384.0)          # distance ~1e6: level clamped to 15
    f["s"] = 1.0
    R = oracle.filter_frame(f, temporal=False)
    assert len(R.gkey) == 1 and R.gcnt[0] == n
    mean = (R.q.sum(0) / n / 2.0 ** 24).astype(np.float32)
    assert np.array_equal(R.out, np.broadcast_to(mean, (n, 3)))


# ------------------------------------------------------------ linear probing
def _random_homes(G, m, rng):
    keys = np.arange(1, G + 1, dtype=np.uint64)
    fps = rng.integers(1, 2**32, G, dtype=np.uint64).astype(np.uint32)
    homes = rng.integers(0, 2**m, G, dtype=np.int64).astype(np.uint32)
    return keys, fps, homes


def test_occupancy_and_displacement_do_not_depend_on_insertion_order():
    rng = np.random.default_rng(5)
    m, G = 10, 700                                  # load 0.68
    keys, fps, homes = _random_homes(G, m, rng)
    base = oracle.simulate_table(keys, fps, homes, m, 1 << m)
    assert base.n_overflow == 0
    for _ in range(100):
        p = rng.permutation(G)
        t = oracle.simulate_table(keys[p], fps[p], homes[p], m, 1 << m)
        assert np.array_equal(t.occupied, base.occupied)
        assert t.total_disp == base.total_disp and t.lmax == base.lmax


def test_occupancy_equals_brute_force_parking():
    """Occupied slots = each home pushed to the first free slot (any order)."""
    rng = np.random.default_rng(6)
    m, G = 7, 90
    keys, fps, homes = _random_homes(G, m, rng)
    occ = np.zeros(1 << m, bool)
    for h in homes:
        s = int(h)
        while occ[s]:
            s = (s + 1) % (1 << m)
        occ[s] = True
    t = oracle.simulate_table(keys, fps, homes, m, 1 << m)
    assert np.array_equal(t.occupied.astype(bool), occ)


@pytest.mark.parametrize("alpha", [0.3, 0.5, 0.7])
def test_mean_displacement_matches_knuth(alpha):
    """Successful search in linear probing takes (1 + 1/(1-a))/2 probes on
    average (Knuth, TAOCP vol. 3, 6.4), i.e. a displacement of
    (1/(1-a) - 1)/2."""
    rng = np.random.default_rng(int(alpha * 10))
    m = 20
    G = int(alpha * (1 << m))
    keys, fps, homes = _random_homes(G, m, rng)
    t = oracle.simulate_table(keys, fps, homes, m, 1 << m)
    want = 0.5 * (1.0 / (1.0 - alpha) - 1.0)
    assert abs(t.total_disp / G - want) / want < 0.04


def test_forced_overflow_fixture():
    """16 slots, one probe step: keys sharing a home overflow after the first."""
    keys = np.array([10, 11, 12, 13], np.uint64)
    fps = np.array([5, 6, 7, 8], np.uint32)
    homes = np.array([3, 3, 3, 9], np.uint32)
    t = oracle.simulate_table(keys, fps, homes, 4, 1)
    assert list(t.gslot) == [3, -1, -1, 9]
    assert t.n_overflow == 2 and t.lmax == 3 and not t.order_free
    t = oracle.simulate_table(keys, fps, homes, 4, 3)
    assert list(t.gslot) == [3, 4, 5, 9] and t.total_disp == 3 and t.n_overflow == 0


def test_forced_fingerprint_alias_fixture():
    keys = np.array([1, 2, 3], np.uint64)
    fps = np.array([77, 77, 77], np.uint32)
    t = oracle.simulate_table(keys, fps, np.array([0, 1, 8], np.uint32), 4, 16)
    assert t.alias and not t.order_free          # keys 1 and 2 share a cluster
    t = oracle.simulate_table(keys, fps, np.array([0, 4, 8], np.uint32), 4, 16)
    assert not t.alias                           # separate clusters never meet


def test_overflowed_vertices_keep_their_own_radiance():
    rng = np.random.default_rng(7)
    f = _frame_arrays(2000, rng)
    f["log2_slots"] = 4; f["max_probe"] = 2; f["s"] = 0.5
    R = oracle.filter_frame(f, temporal=False)
    ovf = (R.flags & oracle.OVERFLOW) != 0
    assert ovf.any() and R.table.n_overflow > 0
    rgb = np.stack([f["r"], f["g"], f["b"]], 1)
    assert np.array_equal(R.out[ovf], rgb[ovf]) and np.all(R.cnt[ovf] == 0)
    assert R.table.occupied.sum() == len(R.gkey) - R.table.n_overflow


# ------------------------------------------------------------ temporal blend
def test_ema_constant_input_stays_constant():
    rng = np.random.default_rng(8)
    c = rng.uniform(0.01, 10, (500, 3)).astype(np.float32)
    keys = np.arange(500, dtype=np.uint64) * 3 + 1
    val = c.copy()
    for _ in range(30):
        val = oracle.temporal_ema(keys, c, keys, val, 0.2)
        assert np.all(np.abs(val - c) <= np.spacing(c) * 2)


@pytest.mark.parametrize("alpha", [0.2, 0.8])
def test_ema_closed_form(alpha):
    """c_T = a^T c_0 + (1 - a) sum_t a^(T-t) c_t for a key seen every frame."""
    rng = np.random.default_rng(9)
    T = 12
    cs = rng.uniform(0.1, 2.0, (T + 1, 64, 3)).astype(np.float32)
    keys = np.arange(64, dtype=np.uint64)
    val = cs[0]
    for t in range(1, T + 1):
        val = oracle.temporal_ema(keys, cs[t], keys, val, alpha)
    a = float(np.float32(alpha))
    want = a ** T * cs[0].astype(np.float64) + sum((1 - a) * a ** (T - t) * cs[t].astype(np.float64)
                                                   for t in range(1, T + 1))
    assert np.allclose(val, want, rtol=2e-6, atol=0)


def test_ema_new_keys_take_the_new_value_and_dropped_keys_vanish():
    keys = np.array([1, 5, 9], np.uint64)
    new = np.array([[1, 1, 1], [2, 2, 2], [3, 3, 3]], np.float32)
    prev_k = np.array([5, 7], np.uint64)
    prev_v = np.array([[10, 10, 10], [20, 20, 20]], np.float32)
    out = oracle.temporal_ema(keys, new, prev_k, prev_v, 0.25)
    b = np.float32(1) - np.float32(0.25)
    assert np.array_equal(out[0], new[0]) and np.array_equal(out[2], new[2])
    assert np.array_equal(out[1], np.float32(0.25) * np.float32(10) + b * np.float32(2) + np.zeros(3, np.float32))


# ------------------------------------------------------------ filter quality
def test_interior_cell_error_matches_lognormal_variance():
    """For a constant truth mu under a mean-one lognormal multiplier, a cell
    of n samples has E[(avg - mu)^2] = mu^2 (exp(sigma^2) - 1) / n."""
    rng = np.random.default_rng(10)
    n = 200000
    sigma, mu = 1.0, 0.7
    f = _frame_arrays(n, rng, sigma=sigma)
    f["px"] = rng.uniform(0, 3, n).astype(np.float32); f["pz"] = rng.uniform(0, 3, n).astype(np.float32)
    f["py"] = np.zeros(n, np.float32)
    f["nx"][:] = 0; f["ny"][:] = 1; f["nz"][:] = 0
    mult = np.exp(sigma * rng.normal(size=n) - sigma ** 2 / 2)
    f["r"] = (mu * mult).astype(np.float32); f["g"] = f["r"]; f["b"] = f["r"]
    f["cam"] = (1.5, 40.0, 1.5); f["s"] = 0.004        # level 5: h = 0.128, about 550 cells
    R = oracle.filter_frame(f, temporal=False)
    err2 = (R.out[:, 0].astype(np.float64) - mu) ** 2
    pred = mu ** 2 * (np.exp(sigma ** 2) - 1) / R.cnt
    # pooled ratio over all vertices: equals 1 in expectation
    ratio = err2.sum() / pred.sum()
    assert 0.85 < ratio < 1.15, ratio
    unf = ((f["r"].astype(np.float64) - mu) ** 2).mean()
    assert abs(unf / (mu ** 2 * (np.exp(sigma ** 2) - 1)) - 1) < 0.1


def test_key_hashes_match_the_key_builder():
    import synth
    f = synth.generate(synth.get("tiny_64x64"), frame=0)
    K = oracle.build_keys(f["px"], f["py"], f["pz"], f["nx"], f["ny"], f["nz"], f["valid"], f["cam"], f["s"],
                          f["seed"], 0, 14)
    home, fp = oracle.key_hashes(K["key"], 14)
    ok = K["flags"] == 0
    assert np.array_equal(home[ok], K["home"][ok]) and np.array_equal(fp[ok], K["fp"][ok])


def test_filter_keys_equals_filter_frame_on_its_keys():
    import synth
    f = synth.generate(synth.get("tiny_64x64"), frame=2)
    Q = oracle.filter_frame(f, temporal=False)
    R = oracle.filter_keys(Q.key, f["r"].numpy(), f["g"].numpy(), f["b"].numpy(), (Q.flags == 0).astype(np.uint8),
                           f["log2_slots"])
    assert np.array_equal(R.out, Q.out) and np.array_equal(R.gsum, Q.gsum)
    assert np.array_equal(R.table.occupied, Q.table.occupied)


def test_synthetic_keys_have_exactly_the_requested_cells():
    import synth
    d = synth.synthetic_keys(100000, 31337)
    assert len(np.unique(d["key"].numpy())) == 31337
    R = oracle.filter_keys(d["key"].numpy(), d["r"].numpy(), d["g"].numpy(), d["b"].numpy(), d["valid"].numpy(), 16)
    assert len(R.gkey) == 31337 and int(R.gcnt.sum()) == 100000
