"""Pins of the oracle's low-density fallbacks (Section 3.3: neighbourhood
search, and the search for similar normals along a probe run) against facts
fixed outside them: a brute-force pooling over vertex pairs built from the
quantised coordinates, levels and normals of the vertices themselves (not
from the packed keys), the threshold that switches the fallback off, a
constant radiance that every pooled mean must reproduce exactly, and
hand-built key fixtures for the key-range edge and the normal classes."""
import numpy as np
import pytest

import oracle
import synth

F = 24


def _random_frame(n, seed, s):
    return synth.mixed_normals_frame(n, seed, s)


def _vertex_attrs(f):
    """Quantised coordinates, second level of detail and normal class vector of
    every vertex, from the step outputs of key construction and the normals."""
    k = oracle.build_keys(f["px"], f["py"], f["pz"], f["nx"], f["ny"], f["nz"], f["valid"], f["cam"], f["s"],
                          f["seed"], 0, f["log2_slots"], steps=True)
    nrm = np.stack([np.asarray(f[c], np.float32) for c in ("nx", "ny", "nz")], 1)
    cls = np.sign(nrm).astype(np.int64)
    return k["xq"].astype(np.int64), k["lvl"][:, 1].astype(np.int64), cls


def _brute_force(f, R, below, mode):
    """Expected output of every vertex whose voxel has fewer than `below`
    vertices, pooling over vertex pairs."""
    xq, lp, cls = _vertex_attrs(f)
    ok = R.flags == 0
    idx = np.nonzero(ok)[0]
    exp = {}
    for v in idx:
        if R.cnt[v] >= below:
            continue
        same_lod = lp[idx] == lp[v]
        if mode == oracle.CUBE:
            near = np.all(np.abs(xq[idx] - xq[v]) <= 1, 1) & np.all(cls[idx] == cls[v], 1)
        else:
            near = np.all(xq[idx] == xq[v], 1) & ((cls[idx] * cls[v]).sum(1) > 0)
        m = idx[same_lod & near]
        S = [sum(int(x) for x in R.q[m, c]) for c in range(3)]
        exp[v] = np.array([(float(S[c]) * 2.0 ** -F) / len(m) for c in range(3)], np.float32)
    return exp


@pytest.mark.parametrize("mode", [oracle.CUBE, oracle.NORMALS])
@pytest.mark.parametrize("s,below", [(0.01, 4), (0.1, 3), (0.1, 64)])
def test_pooling_matches_brute_force_on_the_small_scene(mode, s, below):
    f = synth.generate(synth.get("tiny_64x64"))
    f["s"] = s
    R = oracle.filter_frame(f, temporal=False, low_density_fallback=(below, mode))
    assert R.table.order_free
    exp = _brute_force(f, R, below, mode)
    assert len(exp) > 50
    for v, e in exp.items():
        assert np.array_equal(R.out[v].view(np.uint32), e.view(np.uint32)), (v, R.out[v], e)


@pytest.mark.parametrize("mode", [oracle.CUBE, oracle.NORMALS])
def test_pooling_matches_brute_force_with_mixed_normals(mode):
    f = _random_frame(3000, 11, s=0.08)
    R = oracle.filter_frame(f, temporal=False, low_density_fallback=(6, mode))
    assert R.table.order_free
    exp = _brute_force(f, R, 6, mode)
    assert len(exp) > 100
    changed = 0
    for v, e in exp.items():
        assert np.array_equal(R.out[v].view(np.uint32), e.view(np.uint32)), (v, R.out[v], e)
        changed += not np.array_equal(e, R.gavg[R.vgroup[v]])
    assert changed > 20      # the fallback pools other voxels for a good share of them


def test_vertices_of_dense_voxels_keep_their_voxel_average():
    f = _random_frame(3000, 12, s=0.08)
    P = oracle.filter_frame(f, temporal=False)
    for mode in (oracle.CUBE, oracle.NORMALS):
        R = oracle.filter_frame(f, temporal=False, low_density_fallback=(5, mode))
        dense = (R.flags == 0) & (R.cnt >= 5)
        assert dense.sum() > 100
        assert np.array_equal(R.out[dense].view(np.uint32), P.out[dense].view(np.uint32))
        assert np.array_equal(R.cnt, P.cnt)          # the lookup's count is the voxel's own


@pytest.mark.parametrize("below", [0, 1])
def test_threshold_at_most_one_switches_the_fallback_off(below):
    f = synth.generate(synth.get("tiny_64x64"))
    P = oracle.filter_frame(f, temporal=False)
    for mode in (oracle.CUBE, oracle.NORMALS):
        R = oracle.filter_frame(f, temporal=False, low_density_fallback=(below, mode))
        assert np.array_equal(R.out.view(np.uint32), P.out.view(np.uint32))


def test_constant_radiance_is_reproduced_exactly():
    f = _random_frame(3000, 13, s=0.05)
    c = np.float32(0.375)                             # c * 2^24 is an integer
    for k in ("r", "g", "b"):
        f[k] = np.full_like(f[k], c)
    for mode in (oracle.CUBE, oracle.NORMALS):
        R = oracle.filter_frame(f, temporal=False, low_density_fallback=(1000, mode))
        ok = R.flags == 0
        assert np.all(R.out[ok] == c)


def _key(x, y, z, lp, code):
    return np.uint64((x + 65536) | ((y + 65536) << 17) | ((z + 65536) << 34) | ((lp + 16) << 51) | (code << 56))


def test_normal_classes_pool_by_positive_dot_product():
    # classes per axis: 1 = positive, 2 = negative, 0 = zero
    px, nx, py, pxy, pxny = 1, 2, 1 << 2, 1 | (1 << 2), 1 | (2 << 2)
    keys = [_key(5, 6, 7, 0, c) for c in (px, nx, py, pxy, pxny)] + [_key(5, 6, 8, 0, px)]
    order = np.argsort(np.array(keys, np.uint64))
    gkey = np.array(keys, np.uint64)[order]
    cnt = np.array([1, 3, 4, 2, 5, 7], np.uint32)[order]
    sums = (np.arange(6 * 3, dtype=np.int64).reshape(6, 3) * (1 << 20) + 12345)[order]
    gval = np.zeros((6, 3), np.float32)
    placed = np.ones(6, np.uint8)
    out, pooled = oracle.low_density(gkey, cnt, sums, placed, gval, 2, oracle.NORMALS, F)
    g = int(np.nonzero(gkey == keys[0])[0][0])
    assert pooled.tolist() == [i == g for i in range(6)]
    # +x pools itself, +x+y and +x-y (dot 1); not -x (dot -1), +y (dot 0) or another position
    mine = [gkey.tolist().index(int(k)) for k in (keys[0], keys[3], keys[4])]
    S = sums[mine].sum(0)
    N = int(cnt[mine].sum())
    assert np.array_equal(out[g], np.array([(float(x) * 2.0 ** -F) / N for x in S], np.float32))
    # an unplaced neighbour is not pooled
    placed2 = placed.copy()
    placed2[mine[1]] = 0
    out2, _ = oracle.low_density(gkey, cnt, sums, placed2, gval, 2, oracle.NORMALS, F)
    m2 = [mine[0], mine[2]]
    N2 = int(cnt[m2].sum())
    assert np.array_equal(out2[g], np.array([(float(x) * 2.0 ** -F) / N2 for x in sums[m2].sum(0)], np.float32))


def test_cube_skips_coordinates_outside_the_key_range():
    # a voxel at the largest coordinate: its +1 neighbours do not exist; the
    # voxel one step below on every axis is pooled
    k0 = _key(65535, 0, 0, 3, 1)
    k1 = _key(65534, -1, 1, 3, 1)
    k2 = _key(65535, 2, 0, 3, 1)                      # two steps away on y: not a neighbour
    k3 = _key(65535, 0, 0, 4, 1)                      # another level
    keys = np.array(sorted([k0, k1, k2, k3]), np.uint64)
    cnt = np.array([1, 2, 3, 4], np.uint32)
    sums = np.array([[10, 20, 30], [40, 50, 60], [70, 80, 90], [1, 2, 3]], np.int64) << 24
    out, pooled = oracle.low_density(keys, cnt, sums, np.ones(4, np.uint8), np.zeros((4, 3), np.float32), 2,
                                     oracle.CUBE, F)
    g0, g1 = int(np.nonzero(keys == k0)[0][0]), int(np.nonzero(keys == k1)[0][0])
    assert pooled.sum() == 1 and pooled[g0]
    N = int(cnt[g0]) + int(cnt[g1])
    assert np.array_equal(out[g0], ((sums[g0] + sums[g1]).astype(np.float64) * 2.0 ** -F / N).astype(np.float32))
