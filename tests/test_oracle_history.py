"""Pins of the oracle's history with eviction by priority (Section 3.4.3)
against facts fixed outside it: with max_age 0 and no two voxels of a frame
in one slot it is exactly the two-set moving average; a voxel absent for a
frame is found again two frames later (the closed form of the blend); a
fresh voxel displaces an older one in its slot whatever their counts; among
voxels of the same age the one with more samples stays; voxels older than
max_age vanish; and the result does not depend on the order in which a
frame's voxels are offered."""
import numpy as np
import pytest

import oracle
import synth

ALPHA = 0.2


def _frames(n, w=96, h=64):
    wl = synth.get("hd_1080p_x3")
    for k in range(n):
        f = synth.generate(wl, frame=k, width=w, height=h)
        f["log2_slots"] = 16
        yield {k2: (v.numpy() if hasattr(v, "numpy") else v) for k2, v in f.items()}


def _hslot(keys, log2):
    return np.array([oracle.fmix64(int(k)) & ((1 << log2) - 1) for k in keys], np.uint64)


def test_max_age_zero_without_collisions_is_the_two_set_moving_average():
    H = oracle.History.empty(24, 0)
    state = None
    for k, f in enumerate(_frames(5, 48, 32)):
        R = oracle.filter_frame(f, prev_state=state, temporal=True, alpha_old=ALPHA)
        placed = R.table.gslot >= 0
        assert len(np.unique(_hslot(R.gkey[placed], 24))) == placed.sum()   # no two voxels share a slot
        Rh = oracle.filter_frame(f, temporal=True, alpha_old=ALPHA, history=H, frame=k)
        assert np.array_equal(Rh.out.view(np.uint32), R.out.view(np.uint32))
        assert H.occupied().sum() == placed.sum()
        state = R.state


def test_a_voxel_absent_for_a_frame_is_found_again():
    fa, fb = list(_frames(1))[0], list(_frames(9))[8]   # frame 8: the camera 8 degrees away
    H = oracle.History.empty(22, 3)
    Ra = oracle.filter_frame(fa, temporal=True, alpha_old=ALPHA, history=H, frame=0)
    Rb = oracle.filter_frame(fb, temporal=True, alpha_old=ALPHA, history=H, frame=1)
    Ra2 = oracle.filter_frame(fa, temporal=True, alpha_old=ALPHA, history=H, frame=2)
    # the two-set blend forgets what frame 1 did not see
    R2 = oracle.filter_frame(fa, prev_state=Rb.state, temporal=True, alpha_old=ALPHA)
    # voxels of frame 0 only, alone in their history slot among both frames' voxels
    pa, pb = Ra.gkey[Ra.table.gslot >= 0], Rb.gkey[Rb.table.gslot >= 0]
    sa, sb = _hslot(pa, 22), _hslot(pb, 22)
    slots, counts = np.unique(np.concatenate([sa, sb]), return_counts=True)
    alone = set(slots[counts == 1].tolist())
    only_a = np.isin(Ra.gkey, pa) & ~np.isin(Ra.gkey, pb)
    only_a &= np.array([int(x) in alone for x in _hslot(Ra.gkey, 22)])
    assert only_a.sum() > 100
    a, b = np.float32(ALPHA), np.float32(1) - np.float32(ALPHA)
    exp = (a * Ra.gval[only_a]) + (b * Ra2.gavg[only_a])   # c_old = frame 0's value, c_new = this frame's average
    assert np.array_equal(Ra2.gval[only_a].view(np.uint32), exp.astype(np.float32).view(np.uint32))
    assert np.array_equal(R2.gval[only_a].view(np.uint32), Ra2.gavg[only_a].view(np.uint32))


def _colliding_keys(log2, count, seed=3):
    """`count` distinct keys that share one slot of a 2^log2 history."""
    rng = np.random.default_rng(seed)
    by_slot = {}
    while True:
        k = int(rng.integers(1, 1 << 50))
        s = oracle.fmix64(k) & ((1 << log2) - 1)
        by_slot.setdefault(s, []).append(k)
        if len(by_slot[s]) == count:
            return np.array(sorted(by_slot[s]), np.uint64)


def _offer(H, keys, counts, frame, order=None):
    keys = np.asarray(keys, np.uint64)
    idx = np.argsort(keys) if order is None else np.asarray(order)
    vals = np.stack([keys.astype(np.float64) % 7, np.ones(len(keys)), np.zeros(len(keys))], 1).astype(np.float32)
    oracle.history_update(H, keys[idx], vals[idx], np.asarray(counts, np.uint32)[idx], frame)


def _resident(H):
    return set(int(k) for k in H.key[H.occupied()])


def test_a_fresh_voxel_displaces_an_older_one_whatever_the_counts():
    a, b = _colliding_keys(4, 2)
    H = oracle.History.empty(4, 10)
    _offer(H, [a], [1 << 20], 0)
    _offer(H, [b], [1], 1)
    assert _resident(H) == {int(b)}


def test_more_samples_stay_among_voxels_of_the_same_age():
    keys = _colliding_keys(4, 3)
    for winner in range(3):
        counts = [2] * 3
        counts[winner] = 64
        H = oracle.History.empty(4, 10)
        _offer(H, keys, counts, 0)
        assert _resident(H) == {int(keys[winner])}


def test_voxels_older_than_max_age_vanish():
    H = oracle.History.empty(10, 2)
    keys = np.arange(1, 200, dtype=np.uint64) * np.uint64(2654435761)
    _offer(H, keys, np.full(len(keys), 5), 0)
    n0 = H.occupied().sum()
    _offer(H, np.zeros(0, np.uint64), [], 2)
    assert H.occupied().sum() == n0
    _offer(H, np.zeros(0, np.uint64), [], 3)
    assert H.occupied().sum() == 0


def test_offer_order_does_not_matter():
    rng = np.random.default_rng(4)
    keys = np.unique(rng.integers(1, 1 << 40, 3000).astype(np.uint64))
    counts = rng.integers(1, 300, len(keys))
    results = []
    for trial in range(3):
        H = oracle.History.empty(10, 4)
        for frame in range(3):
            sub = rng.permutation(len(keys))[:1500] if trial == 0 else None
            take = np.arange(len(keys)) if sub is None else np.sort(sub)
            order = rng.permutation(len(take))
            _offer(H, keys[take], counts[take], frame, order=np.argsort(keys[take])[order])
        results.append((H.word.copy(), H.key.copy(), H.stamp.copy()))
    # trials 1 and 2 offered the same voxels in different orders
    for a, b in zip(results[1], results[2]):
        assert np.array_equal(a, b)
