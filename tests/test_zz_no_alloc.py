"""The insert without a workspace argument (pf_build_keys_insert_binned_noalloc)
against the insert that takes one (pf_build_keys_insert_binned), through the
C ABI: two calls in a row on the library's shared scratch, the first large
enough to go through it in two batches, the second smaller.  Keys, flags and
the table's order-free facts (occupied slots, every cell's key, count and
sums) are compared bit for bit; the slot a vertex receives may differ where
keys share a probe run (arrival order), so each vertex's slot is checked to
hold its own key instead."""
import numpy as np
import pytest
import torch

import paper_1902_05942_amd as pf
import synth
from gpu_util import assert_bits_equal, table_contents, to_dev

pytestmark = pytest.mark.gpu


def _run(f, g, noalloc):
    n = g["px"].numel()
    t = pf.Table(f["log2_slots"])
    pf.table_init(t)
    key = torch.empty(n, dtype=torch.int64, device="cuda")
    fl = torch.empty(n, dtype=torch.uint8, device="cuda")
    slot = torch.empty(n, dtype=torch.int32, device="cuda")
    args = (t, g["px"], g["py"], g["pz"], g["nx"], g["ny"], g["nz"], g["valid"], f["cam"], f["s"], f["seed"], 0,
            g["r"], g["g"], g["b"], key, fl, slot)
    if noalloc:
        pf.build_keys_insert_binned_noalloc(*args)
    else:
        ws = torch.empty(pf.insert_workspace_bytes(n, f["log2_slots"]), dtype=torch.uint8, device="cuda")
        pf.build_keys_insert_binned(*args, ws)
    torch.cuda.synchronize()
    return t, key.cpu().numpy().view(np.uint64), fl.cpu().numpy(), slot.cpu().numpy().view(np.uint32)


def test_noalloc_insert_equals_the_workspace_insert(gpu):
    wl = synth.get("hd_1080p_x3")
    # 960 x 540 x 3 = 1,555,200 slots: two batches of the scratch; then
    # 200 x 113 x 3 = 67,800 slots, one batch, a ragged tail of chunks
    for (w, h, frame) in ((960, 540, 2), (200, 113, 5)):
        f = synth.generate(wl, frame=frame, width=w, height=h)
        f["log2_slots"] = 21 if w > 500 else 17
        g = to_dev(f)
        n = g["px"].numel()
        if w > 500:
            assert n > pf.NOALLOC_BATCH
        print(f"noalloc vs workspace insert: {w}x{h}x3 = {n} slots, 2^{f['log2_slots']}-slot table", flush=True)
        ta, ka, fa, sa = _run(f, g, noalloc=True)
        tb, kb, fb, sb = _run(f, g, noalloc=False)
        assert_bits_equal(ka, kb, "keys")
        assert_bits_equal(fa, fb, "flags")
        ok = fa == 0
        assert ok.sum() > 1000
        assert np.array_equal(sa == 0xFFFFFFFF, ~ok)
        ca, cb = table_contents(ta), table_contents(tb)
        assert_bits_equal(ca["occupied"], cb["occupied"], "occupied slots")
        for name in ("key", "count", "sum", "fp"):
            assert_bits_equal(ca[name][np.argsort(ca["key"])], cb[name][np.argsort(cb["key"])], f"table {name}")
        # every filtered vertex's slot holds its own key, in both tables
        for t, s in ((ta, sa), (tb, sb)):
            keys = t.keys().cpu().numpy().view(np.uint64)
            assert_bits_equal(keys[s[ok]], ka[ok], "key at the vertex's slot")
        sta, stb = pf.read_stats(ta), pf.read_stats(tb)
        for k in (pf.STAT_USED, pf.STAT_DISP, pf.STAT_OVERFLOW):
            assert int(sta[k]) == int(stb[k])


def test_noalloc_rejects_what_it_cannot_hold(gpu):
    wl = synth.get("tiny_64x64")
    f = synth.generate(wl, frame=0)
    g = to_dev(f)
    n = g["px"].numel()
    t = pf.Table(26)                                  # above the binned insert's 2^25 slots
    key = torch.empty(n, dtype=torch.int64, device="cuda")
    fl = torch.empty(n, dtype=torch.uint8, device="cuda")
    slot = torch.empty(n, dtype=torch.int32, device="cuda")
    with pytest.raises(pf.PfError):
        pf.build_keys_insert_binned_noalloc(t, g["px"], g["py"], g["pz"], g["nx"], g["ny"], g["nz"], g["valid"],
                                            f["cam"], f["s"], f["seed"], 0, g["r"], g["g"], g["b"], key, fl, slot)
    del t
