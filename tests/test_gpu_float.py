"""GPU parity of the binary32-sum variant (the paper's own accumulation:
one floating-point atomic add per component, Section 3.3.1).  Keys, flags,
counts and the table's occupancy are exact; each average is a binary32 sum
in an order fixed by the hardware, divided once, so it must lie within the
worst-case rounding bound of such a sum around the exact cell mean:
  |avg - mean| <= (gamma_{n-1} (1 + u) + u) * sum|x| / n,
  gamma_k = k u / (1 - k u), u = 2^-24,
for any summation order (atomics, LDS pre-sums or both)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1902_05942_amd as pf
import synth
from gpu_util import assert_bits_equal, gpu_frame, table_contents, to_dev

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


def _frame(case):
    if case == "tiny":
        return synth.generate(synth.get("tiny_64x64"), frame=0)
    if case == "scaled_ragged":
        return synth.generate(synth.get("hd_1080p_x3"), frame=2, width=401, height=229)
    return synth.generate(synth.get("hd_1080p_x3"), frame=0)


@pytest.mark.parametrize("case,agg", [("tiny", 0), ("tiny", 64), ("scaled_ragged", 0), ("scaled_ragged", 256),
                                      ("hd_full", 64)])
def test_float_sums_within_the_summation_bound(gpu, case, agg):
    f = _frame(case)
    n = f["px"].numel()
    print(f"[float] {case} agg={agg} n={n}", flush=True)
    g = to_dev(f)
    t = pf.Table(f["log2_slots"], f["max_probe"], f["frac_bits"], sum_format=pf.SUMS_FLOAT32)
    pf.table_init(t)
    res = gpu_frame(f, g, t, agg=agg)
    R = oracle.float_filter_frame(f)
    assert R.table.order_free
    assert_bits_equal(res["key"], R.key, "keys")
    assert_bits_equal(res["flags"], R.flags, "flags")
    sel = R.vgroup >= 0
    want_cnt = np.where(sel, R.gcnt[np.maximum(R.vgroup, 0)], 0).astype(np.uint32)
    assert_bits_equal(res["cnt"], want_cnt, "counts")
    tc = table_contents(t)
    assert_bits_equal(tc["occupied"], R.table.occupied, "occupancy")
    assert np.array_equal(np.sort(tc["key"]), R.gkey)
    # the high word of every float sum stays zero
    assert np.all((tc["sum"].view(np.uint64) >> np.uint64(32)) == 0)
    # flagged vertices keep their contribution exactly
    own = np.stack([np.asarray(f[c].numpy(), np.float32) for c in ("r", "g", "b")], 1)
    assert_bits_equal(res["out"][~sel], own[~sel], "unfiltered vertices")
    # filtered vertices: within the worst-case bound of a binary32 sum in any order
    gi = R.vgroup[sel]
    cnt = R.gcnt[gi].astype(np.float64)[:, None]
    k = cnt - 1
    gamma = k * U / (1 - k * U)
    bound = (gamma * (1 + U) + U) * R.gabs[gi] / cnt + 2.0 ** -60
    got = res["out"][sel].astype(np.float64)
    mean = R.gmean[gi]
    err = np.abs(got - mean)
    assert np.all(err <= bound), f"{int((err > bound).sum())} averages outside the bound"
    rel = err[mean > 0] / mean[mean > 0]
    p999, mx = float(np.quantile(rel, 0.999)), float(rel.max())
    print(f"[float] {case}: relative error p99.9 {p999:.3g}, max {mx:.3g}, largest cell {int(R.gcnt.max())}")
    assert p999 <= 1e-5


def test_float_tables_are_refused_by_the_multi_view_launch(gpu):
    wl = synth.get("tiny_64x64")
    f = synth.generate(wl, frame=0)
    g = {k: (v.cuda() if torch.is_tensor(v) else v) for k, v in f.items()}
    mvf = pf.MultiViewFilter([(f["px"].numel(), f["log2_slots"])], temporal=False)
    d = mvf.descriptors([g])
    d[0].cur.sum_format = pf.SUMS_FLOAT32
    with pytest.raises(pf.PfError):
        pf.filter_views(d, 256, 0, mvf.ws)
