"""Pins of the oracle's key construction (Algorithm 1) against facts fixed
outside the oracle: published generator outputs, closed forms and exact
invariants of the jitter and quantisation, and brute-force grouping by the
voxel characteristic function of Eq. (7)."""
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLD, name)) as fh:
        return [int(l, 16) for l in fh if l.strip() and not l.startswith("#")]


# ------------------------------------------------------------ generators
def test_pcg32_published_outputs():
    want = _golden("pcg32_seed42_stream54.txt")
    got = [int(x) for x in oracle.pcg32_outputs(42, 54, len(want))]
    assert got == want


def test_splitmix64_published_outputs():
    want = _golden("splitmix64_seed0.txt")
    gamma = 0x9E3779B97F4A7C15
    got = [oracle.splitmix64((k * gamma) % 2**64) for k in range(len(want))]
    assert got == want


def _inv_fmix64(h):
    """Inverse of MurmurHash3's fmix64 from its published constants."""
    M = 2**64
    def unxorshift33(x):
        return x ^ (x >> 33)          # shift >= 32: one application inverts
    c1inv = pow(0xFF51AFD7ED558CCD, -1, M)
    c2inv = pow(0xC4CEB9FE1A85EC53, -1, M)
    h = unxorshift33(h)
    h = (h * c2inv) % M
    h = unxorshift33(h)
    h = (h * c1inv) % M
    return unxorshift33(h)


def test_fmix64_is_the_published_bijection():
    rng = np.random.default_rng(5)
    for k in [0, 1, 2**63, 2**64 - 1] + [int(x) for x in rng.integers(0, 2**63, 200, dtype=np.int64)]:
        assert _inv_fmix64(oracle.fmix64(k)) == k
    # avalanche: one flipped input bit flips about half of the output bits
    flips = [bin(oracle.fmix64(k) ^ oracle.fmix64(k ^ (1 << b))).count("1")
             for k in range(1, 200, 7) for b in range(64)]
    assert 30.0 < np.mean(flips) < 34.0


# ------------------------------------------------------------ level of detail
@pytest.mark.parametrize("k", list(range(-15, 16)))
def test_lod_at_powers_of_four(k):
    cam = (0.0, 0.0, 0.0)
    x = np.float32(2.0) ** k                     # d = 2^k, d^2 = 4^k exactly
    assert oracle.level_of_detail(cam, x, 0, 0) == k
    below = np.nextafter(x, np.float32(0))       # d^2 rounds below 4^k
    assert oracle.level_of_detail(cam, below, 0, 0) == k - 1
    # d^2 = 2 * 4^k: still level k (floor of log2 d = k + 1/2)
    assert oracle.level_of_detail(cam, x, x, 0) == k


def test_lod_clamps_and_zero_distance():
    assert oracle.level_of_detail((1, 2, 3), 1, 2, 3) == -16
    assert oracle.level_of_detail((0, 0, 0), 2.0 ** -40, 0, 0) == -16
    assert oracle.level_of_detail((0, 0, 0), 2.0 ** 40, 0, 0) == 15
    assert oracle.level_of_detail((0, 0, 0), 3e38, 3e38, 0) == 15     # d^2 overflows to inf


def test_lod_is_monotone_in_distance():
    ds = np.sort(np.random.default_rng(1).uniform(1e-3, 1e4, 5000).astype(np.float32))
    ls = [oracle.level_of_detail((0, 0, 0), d, 0, 0) for d in ds]
    assert all(a <= b for a, b in zip(ls, ls[1:]))
    for d, l in zip(ds[::97], ls[::97]):
        assert 2.0 ** l <= d < 2.0 ** (l + 1)


# ------------------------------------------------------------ jitter
def _keys(pos, nrm, cam=(0.0, 0.0, -50.0), s=0.01, seed=7, m=14, steps=True, idx_base=0):
    pos = np.asarray(pos, np.float32); nrm = np.asarray(nrm, np.float32)
    return oracle.build_keys(pos[:, 0], pos[:, 1], pos[:, 2], nrm[:, 0], nrm[:, 1], nrm[:, 2], None,
                             cam, s, seed, idx_base, m, steps=steps)


def _rand_unit(n, rng):
    v = rng.normal(size=(n, 3))
    return (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)


@pytest.mark.parametrize("axis,sign", [(a, s) for a in range(3) for s in (1.0, -1.0)])
def test_jitter_axis_normal_is_exactly_tangent(axis, sign):
    """For n = +-e_axis the normal component of the jitter is exactly zero."""
    rng = np.random.default_rng(axis * 2 + (sign > 0))
    n = 4000
    pos = rng.uniform(-3, 3, (n, 3)).astype(np.float32)
    nrm = np.zeros((n, 3), np.float32); nrm[:, axis] = sign
    k = _keys(pos, nrm)
    assert np.array_equal(k["xj"][:, axis], pos[:, axis])
    # tangent offsets are r * h with r in [-1/2, 1/2): |x' - x| <= h/2
    h = (0.01 * np.exp2(k["lvl"][:, 0].astype(np.float64)))[:, None]
    off = (k["xj"].astype(np.float64) - pos.astype(np.float64))
    t_axes = [c for c in range(3) if c != axis]
    assert np.all(np.abs(off[:, t_axes]) <= 0.5 * h * (1 + 1e-6) + 1e-6)


def test_jitter_moments_are_uniform_cell_wide():
    """Tangential offsets are uniform on [-h/2, h/2): mean 0, variance h^2/12."""
    rng = np.random.default_rng(3)
    n = 60000
    pos = np.zeros((n, 3), np.float32); pos[:, 0] = rng.uniform(0.5, 0.9, n)
    nrm = np.zeros((n, 3), np.float32); nrm[:, 1] = 1.0
    k = _keys(pos, nrm, cam=(0.0, 0.0, -100.0))   # every vertex at level 6
    assert np.all(k["lvl"][:, 0] == 6)
    h = 0.01 * 64
    for c in (0, 2):
        u = (k["xj"][:, c].astype(np.float64) - pos[:, c]) / h
        assert abs(u.mean()) < 0.005
        assert abs(u.var() - 1.0 / 12.0) < 0.002
        assert u.min() >= -0.5 - 1e-6 and u.max() < 0.5 + 1e-6 and u.min() < -0.49 and u.max() > 0.49


def test_jitter_generic_normal_stays_in_tangent_plane():
    rng = np.random.default_rng(11)
    n = 5000
    pos = rng.uniform(-2, 2, (n, 3)).astype(np.float32)
    nrm = _rand_unit(n, rng)
    k = _keys(pos, nrm)
    h = 0.01 * np.exp2(k["lvl"][:, 0].astype(np.float64))
    off = (k["xj"].astype(np.float64) - pos.astype(np.float64)) / h[:, None]
    along_n = np.abs((off * nrm).sum(1))
    assert along_n.max() < 1e-3                 # zero up to binary32 rounding
    assert np.abs(off).max() < 0.87             # |r - (r.n)n| <= |r| <= sqrt(3)/2


def test_jitter_depends_on_seed_and_vertex_index():
    pos = np.tile(np.array([[0.3, 0.0, 0.2]], np.float32), (64, 1))
    nrm = np.tile(np.array([[0.0, 1.0, 0.0]], np.float32), (64, 1))
    a = _keys(pos, nrm, seed=1)["xj"]
    b = _keys(pos, nrm, seed=2)["xj"]
    c = _keys(pos, nrm, seed=1, idx_base=64)["xj"]
    assert len({tuple(x) for x in a}) == 64     # each vertex index draws its own jitter
    assert not np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.array_equal(a, _keys(pos, nrm, seed=1)["xj"])


# ------------------------------------------------------------ quantisation
def test_cell_centres_quantise_to_their_cell():
    """x = (k + 1/2) h with a tangent jitter of at most h/2 stays in cell k."""
    rng = np.random.default_rng(2)
    n = 3000
    cam = (0.0, 0.0, -100.0)                     # distance in [64, 128): level 6
    h = np.float32(0.01) * np.float32(64)
    kx = rng.integers(-20, 20, n); kz = rng.integers(-20, 20, n)
    pos = np.stack([(kx + 0.5) * h, np.zeros(n), (kz + 0.5) * h], 1).astype(np.float32)
    nrm = np.tile(np.array([[0.0, 1.0, 0.0]], np.float32), (n, 1))
    k = _keys(pos, nrm, cam=cam)
    assert np.all(k["lvl"] == 6)
    assert np.array_equal(k["xq"][:, 0], kx) and np.array_equal(k["xq"][:, 2], kz)
    assert np.all(k["xq"][:, 1] == 0)


def test_quantisation_uses_the_level_at_the_jittered_point():
    """Just inside distance 2^7 (level 6) with x-jitter of +-h/2: vertices whose
    jittered point crosses 128 quantise with h = s 2^7, the others with s 2^6."""
    n = 4000
    s = np.float32(0.125)
    x0 = np.float32(128.0) - np.float32(2.0)      # level 6, h = 8: x' in [122, 130)
    pos = np.stack([np.full(n, x0), np.zeros(n), np.zeros(n)], 1).astype(np.float32)
    nrm = np.tile(np.array([[0.0, 0.0, 1.0]], np.float32), (n, 1))   # jitter in x and y
    k = _keys(pos, nrm, cam=(0.0, 0.0, 0.0), s=s)
    assert np.all(k["lvl"][:, 0] == 6)
    lp = k["lvl"][:, 1]
    assert set(np.unique(lp)) == {6, 7}
    # The y-jitter (at most 4) lengthens d by at most 16/256, so level 7 means
    # x' >= 127.9: floor(x'/16) is 8, or 7 in the sliver [127.9, 128).
    # Level 6 means x' < 128: floor(x'/8) = 15.  Quantising with l instead of
    # l' would give 16 for every x' >= 128.
    q7 = k["xq"][lp == 7, 0]
    assert np.all((q7 == 8) | (q7 == 7)) and (q7 == 8).mean() > 0.9
    assert np.all(k["xq"][lp == 6, 0] == 15)
    assert np.all(k["xj"][lp == 7, 0] >= 127.9)


def test_keyrange_flag():
    pos = np.array([[0.5, 0.0, 0.5], [2.0e7, 0.0, 0.0], [-3.0e7, 0.0, 0.0]], np.float32)
    nrm = np.array([[0, 1, 0]] * 3, np.float32)
    k = _keys(pos, nrm, cam=(0.0, 0.0, 0.0))
    # level is clamped at 15: h = 327.68, |x~| reaches 2^16 beyond about 2.1e7
    assert list(k["flags"]) == [0, 0, oracle.KEYRANGE]
    assert k["key"][2] == 0 and k["fp"][2] == 0


def key_range_boundary_frame():
    """Vertices whose x'/h lands exactly on either side of +-2^16 (x~ = floor(x'/h)).

    With s = 1.5 * 2^-16, a vertex at X = m * s * 2^k on the x axis (camera at
    the origin) lies at distance 1.5 * 2^k * m / 2^16, so its level is k for
    m near 2^16; its normal +x makes the jitter's x component exactly zero, so
    x'/h = m exactly and x~ = floor(m).  Returns (pos, nrm, s, expected x~ or
    None where the key cannot hold it, |x~| >= 2^16)."""
    s = 1.5 * 2.0 ** -16
    ms = [-65536.5, -65536.0, -65535.5, -65535.0, -65534.5, 65534.5, 65535.0, 65535.5, 65536.0, 65536.5]
    pos, want = [], []
    for k in (-3, 0, 5):
        for m in ms:
            x = m * s * 2.0 ** k
            assert float(np.float32(x)) == x           # exact: at most 19 significant bits
            pos.append([x, 0.0, 0.0])
            q = int(np.floor(m))
            want.append(q if -65536 < q < 65536 else None)
    nrm = np.tile(np.array([[1.0, 0.0, 0.0]], np.float32), (len(pos), 1))
    return np.array(pos, np.float32), nrm, s, want


def test_key_range_boundary_is_symmetric():
    """|x~| < 2^16 (reading of Algorithm 1's quantisation with a 17-bit field
    per coordinate): x'/h in [-2^16, -2^16 + 1) is out of range like
    [2^16, 2^16 + 1), while -65535 and 65535 are the extreme cells kept."""
    pos, nrm, s, want = key_range_boundary_frame()
    k = _keys(pos, nrm, cam=(0.0, 0.0, 0.0), s=s)
    lv = np.repeat([-3, 0, 5], len(want) // 3)
    assert np.array_equal(k["lvl"][:, 0], lv) and np.array_equal(k["lvl"][:, 1], lv)
    for i, q in enumerate(want):
        if q is None:
            assert k["flags"][i] == oracle.KEYRANGE and k["key"][i] == 0, (i, pos[i, 0])
        else:
            assert k["flags"][i] == 0, (i, pos[i, 0])
            assert _unpack(k["key"][i])[0] == q and _unpack(k["key"][i])[3] == lv[i]
    assert sum(q is None for q in want) == 15 and {-65535, 65535} <= {q for q in want if q is not None}


def test_invalid_inputs_are_flagged():
    pos = np.array([[0.5, 0, 0.5], [np.nan, 0, 0], [0.5, 0, 0.5], [0.5, 0, np.inf]], np.float32)
    nrm = np.array([[0, 1, 0], [0, 1, 0], [0, np.nan, 0], [0, 1, 0]], np.float32)
    k = oracle.build_keys(pos[:, 0], pos[:, 1], pos[:, 2], nrm[:, 0], nrm[:, 1], nrm[:, 2],
                          np.array([1, 1, 1, 1], np.uint8), (0, 0, -5), 0.01, 1, 0, 10)
    assert list(k["flags"]) == [0, 1, 1, 1]
    k = oracle.build_keys(pos[:1, 0], pos[:1, 1], pos[:1, 2], nrm[:1, 0], nrm[:1, 1], nrm[:1, 2],
                          np.array([0], np.uint8), (0, 0, -5), 0.01, 1, 0, 10)
    assert k["flags"][0] == oracle.INVALID


# ------------------------------------------------------------ key layout and hashes
def _unpack(K):
    K = int(K)
    q = [((K >> (17 * c)) & 0x1FFFF) - 65536 for c in range(3)]
    return (*q, ((K >> 51) & 31) - 16, (K >> 56) & 63, K >> 62)


def test_normal_classes_and_key_fields():
    nrm = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                    [0.6, -0.8, 0], [-0.0, 0.6, -0.8], [0.577, 0.577, 0.577]], np.float32)
    want = [1, 2, 4, 8, 16, 32, 1 | 8, 4 | 32, 1 | 4 | 16]
    n = len(nrm)
    pos = np.tile(np.array([[0.3, 0.1, 0.2]], np.float32), (n, 1))
    k = _keys(pos, nrm)
    for i in range(n):
        qx, qy, qz, lv, code, top = _unpack(k["key"][i])
        assert code == want[i]
        assert (qx, qy, qz) == tuple(k["xq"][i]) and lv == k["lvl"][i, 1] and top == 0


def test_brute_force_voxel_partition_equals_key_grouping():
    """Eq. (7): vertices share a voxel iff floor(s(k)k) and s(k) agree (and the
    normal class, which is part of the key here).  Brute-force O(n^2) grouping
    of the (x~, l', class) tuples must equal grouping by the packed key."""
    rng = np.random.default_rng(4)
    for s in (0.01, 0.1, 0.5):
        n = 600
        pos = rng.uniform(-2, 2, (n, 3)).astype(np.float32)
        pos[: n // 2, 1] = 0.0
        nrm = np.zeros((n, 3), np.float32)
        nrm[np.arange(n), rng.integers(0, 3, n)] = rng.choice([-1.0, 1.0], n)
        k = _keys(pos, nrm, cam=(0.0, 2.0, -6.0), s=s)
        code = [_unpack(K)[4] for K in k["key"]]
        tup = [tuple(k["xq"][i]) + (k["lvl"][i, 1], code[i]) for i in range(n)]
        same_tuple = np.array([[tup[i] == tup[j] for j in range(n)] for i in range(n)])
        same_key = k["key"][:, None] == k["key"][None, :]
        assert np.array_equal(same_tuple, same_key)
        if s == 0.5:
            assert same_key.sum() > n + 50       # some voxels really are shared


def test_home_ignores_normal_fingerprint_does_not():
    n = 2000
    rng = np.random.default_rng(8)
    pos = rng.uniform(-2, 2, (n, 3)).astype(np.float32); pos[:, 1] = 0.0
    up = np.tile(np.array([[0, 1, 0]], np.float32), (n, 1))
    tilted = np.tile(np.array([[0.6, 0.8, 0.0]], np.float32), (n, 1))   # same jitter plane? no: compare keys only
    a = _keys(pos, up, m=20)
    b = _keys(pos, tilted, m=20)
    same_pos = np.all(a["xq"] == b["xq"], 1) & (a["lvl"][:, 1] == b["lvl"][:, 1])
    assert same_pos.sum() > 100
    assert np.array_equal(a["home"][same_pos], b["home"][same_pos])
    assert np.all(a["fp"][same_pos] != b["fp"][same_pos])
    assert np.all(a["fp"] != 0) and np.all(a["home"] < 2**20)


def test_home_is_uniform_over_slots():
    rng = np.random.default_rng(9)
    n = 200000
    pos = rng.uniform(-50, 50, (n, 3)).astype(np.float32)
    nrm = np.tile(np.array([[0, 0, 1]], np.float32), (n, 1))
    k = _keys(pos, nrm, s=0.001, m=8, steps=False)
    keys, first = np.unique(k["key"], return_index=True)
    counts = np.bincount(k["home"][first], minlength=256)
    expected = len(keys) / 256
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert chi2 < 255 + 5 * np.sqrt(2 * 255)     # 5 sigma of the chi-square with 255 d.o.f.
