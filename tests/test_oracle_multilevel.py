"""Pins of the oracle's multi-level accumulation (Section 3.3.2) against facts
fixed outside it: the coarser voxel's key computed by quantising the jittered
position at the coarser level equals the one derived from the vertex's own
key by halving its cell coordinates (floor division, an identity of IEEE
quotients by powers of two), brute-force means over the vertices that share
the coarser voxel, the threshold that switches the coarser level off, and the
top level of the key's range."""
import numpy as np
import pytest

import oracle
import synth

F = 24
M17 = (1 << 17) - 1


def _derived_coarse(key, flags, k):
    """Key of the voxel k levels up, from the key's fields."""
    out = np.zeros_like(key)
    for i in np.nonzero(flags == 0)[0]:
        K = int(key[i])
        x = [((K >> (17 * c)) & M17) - 65536 for c in range(3)]
        lp = ((K >> 51) & 31) - 16 + k
        if lp > 15:
            continue
        y = [v >> k for v in x]  # Python's >> floors negative values
        out[i] = (y[0] + 65536) | ((y[1] + 65536) << 17) | ((y[2] + 65536) << 34) | ((lp + 16) << 51) | \
                 ((K >> 56) << 56)
    return out


def _frames():
    tiny = synth.generate(synth.get("tiny_64x64"))
    scaled = synth.generate(synth.get("hd_1080p_x3"), frame=3, width=160, height=90)
    cloud = synth.mixed_normals_frame(3000, 5, 0.03)
    for f in (tiny, scaled, cloud):
        yield {k: (v.numpy() if hasattr(v, "numpy") else v) for k, v in f.items()}


@pytest.mark.parametrize("k", [1, 2, 3])
def test_coarse_key_equals_halved_cell_coordinates(k):
    for f in _frames():
        args = (f["px"], f["py"], f["pz"], f["nx"], f["ny"], f["nz"], f["valid"], f["cam"], f["s"], f["seed"], 0,
                f["log2_slots"])
        fine = oracle.build_keys(*args)
        coarse = oracle.build_keys(*args, level_up=k)
        ok = (fine["flags"] == 0) & (coarse["flags"] == 0)
        assert ok.sum() > 1000
        exp = _derived_coarse(fine["key"], fine["flags"], k)
        assert np.array_equal(coarse["key"][ok], exp[ok])
        # a valid fine key never becomes out of range at a coarser level
        # except through its level field
        lp = (fine["key"].astype(np.uint64) >> np.uint64(51)).astype(np.int64) - 16
        bad = (fine["flags"] == 0) & (coarse["flags"] != 0)
        assert np.all(lp[bad] + k > 15)


def test_coarse_level_beyond_the_key_range_is_flagged():
    f = synth.mixed_normals_frame(500, 6, 0.01)
    f["cam"] = (0.0, 1.0, -1.0e5)   # distances above 2^16: l' clamped to 15 for every vertex
    R = oracle.filter_frame(f, temporal=False, level_up=1)
    fine = oracle.filter_frame(f, temporal=False)
    assert np.all(fine.flags == 0)
    assert np.all(R.flags == oracle.KEYRANGE)
    out, cnt = oracle.multilevel(fine, R, 1 << 30)
    assert np.array_equal(out, fine.out) and np.array_equal(cnt, fine.cnt)


@pytest.mark.parametrize("k,below", [(1, 4), (2, 8)])
def test_multilevel_matches_brute_force(k, below):
    for f in _frames():
        fine = oracle.filter_frame(f, temporal=False)
        R = oracle.filter_frame(f, temporal=False, level_up=k)
        assert fine.table.order_free and R.table.order_free
        out, cnt = oracle.multilevel(fine, R, below)
        kk = oracle.build_keys(f["px"], f["py"], f["pz"], f["nx"], f["ny"], f["nz"], f["valid"], f["cam"], f["s"],
                               f["seed"], 0, f["log2_slots"], steps=True)
        xq, lp = kk["xq"].astype(np.int64), kk["lvl"][:, 1].astype(np.int64)
        cls = np.sign(np.stack([np.asarray(f[c], np.float32) for c in ("nx", "ny", "nz")], 1)).astype(np.int64)
        ok = np.nonzero(fine.flags == 0)[0]
        used = 0
        for v in ok[::3]:
            if fine.cnt[v] >= below or lp[v] + k > 15:
                assert np.array_equal(out[v], fine.out[v]) and cnt[v] == fine.cnt[v]
                continue
            m = ok[np.all((xq[ok] >> k) == (xq[v] >> k), 1) & (lp[ok] == lp[v]) & np.all(cls[ok] == cls[v], 1)]
            S = [sum(int(x) for x in fine.q[m, c]) for c in range(3)]
            e = np.array([(float(S[c]) * 2.0 ** -F) / len(m) for c in range(3)], np.float32)
            assert np.array_equal(out[v].view(np.uint32), e.view(np.uint32)), (v, out[v], e)
            assert cnt[v] == len(m)
            used += 1
        assert used > 30


@pytest.mark.parametrize("below", [0, 1])
def test_threshold_at_most_one_keeps_the_own_level(below):
    for f in _frames():
        fine = oracle.filter_frame(f, temporal=False)
        R = oracle.filter_frame(f, temporal=False, level_up=1)
        out, cnt = oracle.multilevel(fine, R, below)
        assert np.array_equal(out.view(np.uint32), fine.out.view(np.uint32))
        assert np.array_equal(cnt, fine.cnt)
