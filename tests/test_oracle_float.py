"""Pins of the oracle's binary32-sum variant (the paper's own accumulation
with one floating-point atomic add per component, Section 3.3.1): its
partition is the exact group-by already pinned for the fixed-point path, and
its float64 cell sums are checked against independent computations."""
import math

import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def tiny():
    f = synth.generate(synth.get("tiny_64x64"), frame=0)
    return f, oracle.float_filter_frame(f), oracle.filter_frame(f, temporal=False)


def test_partition_equals_the_fixed_point_group_by(tiny):
    f, R, Q = tiny
    assert np.array_equal(R.gkey, Q.gkey) and np.array_equal(R.gcnt, Q.gcnt)
    assert np.array_equal(R.vgroup, Q.vgroup) and np.array_equal(R.flags, Q.flags)
    assert np.array_equal(R.table.occupied, Q.table.occupied)


def test_sums_agree_with_the_fixed_point_sums_within_their_rounding(tiny):
    # each fixed-point term is the contribution rounded to 2^-24: at most 2^-25 off
    f, R, Q = tiny
    d = np.abs(R.gsum - Q.gsum.astype(np.float64) * 2.0 ** -24)
    assert np.all(d <= Q.gcnt[:, None] * 2.0 ** -25 + 1e-12 * R.gabs)


def test_sums_agree_with_exactly_rounded_sums(tiny):
    # math.fsum returns the correctly rounded exact sum of each cell
    f, R, _ = tiny
    rgb = [np.asarray(f[c], np.float32) for c in ("r", "g", "b")]
    members = {}
    for i, gidx in enumerate(R.vgroup):
        if gidx >= 0:
            members.setdefault(int(gidx), []).append(i)
    for gidx, idx in members.items():
        for c in range(3):
            exact = math.fsum(float(rgb[c][i]) for i in idx)
            assert abs(R.gsum[gidx, c] - exact) <= len(idx) * 2.0 ** -53 * R.gabs[gidx, c]
            assert R.gabs[gidx, c] == pytest.approx(math.fsum(abs(float(rgb[c][i])) for i in idx), rel=1e-15)


def test_constant_contributions_average_exactly():
    f = synth.generate(synth.get("tiny_64x64"), frame=1)
    for c, v in (("r", 0.3), ("g", 1.0), ("b", 7.25)):
        f[c] = f[c] * 0 + np.float32(v)
    R = oracle.float_filter_frame(f)
    for c, v in enumerate((0.3, 1.0, 7.25)):
        # n copies of a 24-bit significand sum exactly in float64 (n < 2^29), so the mean is x itself
        assert np.all(R.gmean[:, c] == float(np.float32(v)))


def test_nonfinite_contributions_are_invalid_and_nothing_is_out_of_range():
    f = synth.generate(synth.get("tiny_64x64"), frame=0)
    r = np.asarray(f["r"].numpy(), np.float32).copy()
    valid = np.nonzero(np.asarray(f["valid"]))[0]
    r[valid[0]] = np.nan
    r[valid[1]] = np.float32(3e38)          # far out of the fixed-point range, fine in binary32
    f["r"] = r
    R = oracle.float_filter_frame(f)
    assert R.flags[valid[0]] == oracle.INVALID and R.vgroup[valid[0]] == -1
    assert R.flags[valid[1]] == 0 and R.vgroup[valid[1]] >= 0
    Q = oracle.filter_frame(f, temporal=False)
    assert Q.flags[valid[1]] == oracle.RADRANGE
