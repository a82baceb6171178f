"""Pins of the oracle's temporal lookup across levels (Section 3.4.2:
resolution changes between frames) against facts fixed outside it: where the
key itself is found or nothing is, it equals the two-set blend (moving average
and integration, pinned on their own); hand-built parent and children
fixtures (keys packed here, values dyadic so the count-weighted mean is exact)
follow the stated rules -- the parent's value distributed with an eighth of
its samples, the children's count-weighted mean with the sum of their
counts; the exact key wins over the parent and the parent over the children."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

A = np.float32(0.2)


def _key(x, y, z, lp, code=1):
    return (x + 65536) | ((y + 65536) << 17) | ((z + 65536) << 34) | ((lp + 16) << 51) | (code << 56)


def _blend(c_old, c_new, alpha):
    a = np.float32(alpha)
    return (a * np.float32(c_old)) + ((np.float32(1) - a) * np.float32(c_new))


@pytest.mark.parametrize("mode", [0, 1])
def test_found_or_absent_keys_blend_as_the_two_set_pass(mode):
    wl = synth.get("hd_1080p_x3")
    state = None
    for k in range(4):
        f = synth.generate(wl, frame=k, width=320, height=180)
        f["log2_slots"] = 18
        R = oracle.filter_frame(f, temporal=False)
        pk, pv, pc = state if state else (np.zeros(0, np.uint64), np.zeros((0, 3), np.float32), np.zeros(0, np.uint32))
        v, n, how = oracle.temporal_levels(R.gkey, R.gavg, R.gcnt, pk, pv, pc, mode, A, 40)
        if mode == 0:
            ref, refn = oracle.temporal_ema(R.gkey, R.gavg, pk, pv, A), R.gcnt
        else:
            ref, refn = oracle.temporal_integrate(R.gkey, R.gavg, R.gcnt, pk, pv, pc, 40)
        same = how <= 1
        assert np.array_equal(v[same].view(np.uint32), ref[same].view(np.uint32))
        assert np.array_equal(n[same], refn[same])
        if k:
            assert (how >= 2).sum() > 0      # the orbit changes some voxels' level
        state = (R.gkey, v, n)


def _one(cur, prev, mode=0, new=(0.5, 0.25, 1.0), ncur=3):
    pk = np.array(sorted(k for k, _, _ in prev), np.uint64)
    order = {k: i for i, k in enumerate(pk.tolist())}
    pv = np.zeros((len(pk), 3), np.float32)
    pc = np.zeros(len(pk), np.uint32)
    for k, val, cnt in prev:
        pv[order[k]] = val
        pc[order[k]] = cnt
    gkey = np.array([cur], np.uint64)
    v, n, how = oracle.temporal_levels(gkey, np.array([new], np.float32), np.array([ncur], np.uint32), pk, pv, pc,
                                       mode, A, 1 << 24)
    return v[0], int(n[0]), int(how[0])


def test_parent_value_is_distributed_to_its_child():
    K = _key(5, -3, 7, 2)
    P = _key(2, -2, 3, 3)                       # floor(5/2), floor(-3/2), floor(7/2); level + 1
    new = (0.5, 0.25, 1.0)
    v, n, how = _one(K, [(P, (2.0, 4.0, 8.0), 80)], 0, new)
    assert how == 2 and n == 3
    assert np.array_equal(v, np.array([_blend(c, d, A) for c, d in zip((2.0, 4.0, 8.0), new)], np.float32))
    # integration: an eighth of the parent's samples
    v, n, how = _one(K, [(P, (2.0, 4.0, 8.0), 80)], 1, new)
    assert how == 2 and n == 10 + 3
    al = np.float32(10) / np.float32(13)
    assert np.array_equal(v, np.array([_blend(c, d, al) for c, d in zip((2.0, 4.0, 8.0), new)], np.float32))
    # fewer than 8 samples cannot be spread: not used in integration
    v, n, how = _one(K, [(P, (2.0, 4.0, 8.0), 7)], 1, new)
    assert how == 0 and n == 3 and np.array_equal(v, np.array(new, np.float32))


def test_children_are_added_up():
    K = _key(-4, 6, 0, 0)
    kids = [(_key(2 * -4 + dx, 2 * 6 + dy, 0 + dz, -1), dx, dy, dz) for dx, dy, dz in ((0, 0, 0), (1, 0, 1), (1, 1, 1))]
    vals = [(1.0, 2.0, 0.5), (3.0, 0.25, 4.0), (0.75, 1.5, 2.0)]
    cnts = [4, 1, 3]
    prev = [(k, vv, c) for (k, *_), vv, c in zip(kids, vals, cnts)] + [(_key(100, 0, 0, -1), (9.0, 9.0, 9.0), 5)]
    new = (0.5, 0.25, 1.0)
    for mode in (0, 1):
        v, n, how = _one(K, prev, mode, new)
        assert how == 3
        N = sum(cnts)
        mean = [float(sum(Fraction(c) * Fraction(vv[ch]) for vv, c in zip(vals, cnts)) / N) for ch in range(3)]
        al = A if mode == 0 else np.float32(N) / np.float32(N + 3)
        assert np.array_equal(v, np.array([_blend(m, d, al) for m, d in zip(mean, new)], np.float32))
        assert n == (3 if mode == 0 else N + 3)


def test_exact_before_parent_before_children():
    K = _key(5, 5, 5, 1)
    exact = (K, (1.0, 1.0, 1.0), 2)
    parent = (_key(2, 2, 2, 2), (2.0, 2.0, 2.0), 16)
    child = (_key(10, 10, 10, 0), (4.0, 4.0, 4.0), 3)
    assert _one(K, [exact, parent, child])[2] == 1
    assert _one(K, [parent, child])[2] == 2
    assert _one(K, [child])[2] == 3
    assert _one(K, [])[2] == 0


def test_children_are_summed_in_the_stated_order():
    # count-weighted terms 2^60, 1, -2^60 at j = 0 (origin), 1 (dx), 2 (dy):
    # summed in that order the 1 is lost in double, in any order putting the
    # two large terms first it is kept
    K = _key(3, 3, 3, 0)
    big = np.float32(2.0 ** 40)
    prev = [(_key(6, 6, 6, -1), (big, big, big), 1 << 20), (_key(7, 6, 6, -1), (1.0, 1.0, 1.0), 1),
            (_key(6, 7, 6, -1), (-big, -big, -big), 1 << 20)]
    v, n, how = _one(K, prev, 1, (0.0, 0.0, 0.0), ncur=1)
    assert how == 3
    assert np.all(v == 0.0)
