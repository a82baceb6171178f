"""GPU parity of multi-level accumulation (pf_coarsen_keys, a second table,
pf_query_multilevel) against the CPU oracle, bit for bit: coarse keys and
flags, the coarse table, and the combined lookup, on the small scene, a
scaled frame with a ragged tail, the full 1080p x3 frame (fused insert), and
four frames of the moving average through FrameFilter."""
import numpy as np
import pytest
import torch

import oracle
import paper_1902_05942_amd as pf
import synth
from gpu_util import assert_bits_equal, check_frame_against_oracle, gpu_frame, to_dev

pytestmark = pytest.mark.gpu


def _host(f):
    return {k: (v.cpu() if torch.is_tensor(v) else v) for k, v in f.items()}


def _case(case):
    if case == "tiny":
        return synth.generate(synth.get("tiny_64x64")), 64
    if case == "scaled_ragged":
        return synth.generate(synth.get("hd_1080p_x3"), frame=2, width=401, height=229), "binned"
    return synth.generate(synth.get("hd_1080p_x3"), frame=0, device="cuda"), "fused"


@pytest.mark.parametrize("case,levels,below", [("tiny", 1, 4), ("tiny", 2, 64), ("scaled_ragged", 2, 8),
                                               ("hd_full", 1, 4)])
def test_multilevel_bit_exact(gpu, case, levels, below):
    f, agg = _case(case)
    n = len(f["px"])
    print(f"[multilevel] {case} levels={levels} below={below} n={n}", flush=True)
    g = to_dev(f)
    fine = pf.Table(f["log2_slots"], f["max_probe"], f["frac_bits"])
    coarse = pf.Table(f["log2_slots"], f["max_probe"], f["frac_bits"])
    pf.table_init(fine)
    pf.table_init(coarse)
    res = gpu_frame(f, g, fine, agg=agg, want_fp_home=False)
    Rf = oracle.filter_frame(_host(f), temporal=False)
    check_frame_against_oracle(res, Rf, fine)
    dev = g["px"].device
    key = torch.from_numpy(res["key"].view(np.int64)).to(dev)
    vflags = torch.from_numpy(res["flags"]).to(dev)
    slot = torch.from_numpy(res["slot"].view(np.int32)).to(dev)
    key_c = torch.empty_like(key)
    vflags_c = torch.empty_like(vflags)
    slot_c = torch.empty_like(slot)
    pf.clear(coarse)
    pf.coarsen_keys(key, vflags, levels, key_c, vflags_c)
    ws = torch.empty(pf.insert_workspace_bytes(n, coarse.log2_slots), dtype=torch.uint8, device=dev)
    pf.insert_accumulate_binned(coarse, key_c, g["r"], g["g"], g["b"], vflags_c, slot_c, ws)
    out = tuple(torch.empty_like(g["r"]) for _ in range(3))
    cnt = torch.empty(n, dtype=torch.int32, device=dev)
    pf.query_multilevel(fine, coarse, slot, slot_c, g["r"], g["g"], g["b"], vflags, vflags_c, below, False,
                        out[0], out[1], out[2], cnt)
    torch.cuda.synchronize()
    Rc = oracle.filter_frame(_host(f), temporal=False, level_up=levels)
    assert Rc.table.order_free
    fl_c = vflags_c.cpu().numpy()
    assert_bits_equal(fl_c, Rc.flags, "coarse flags")
    ok = Rc.flags == 0
    assert_bits_equal(key_c.cpu().numpy().view(np.uint64)[ok], Rc.key[ok], "coarse keys")
    exp_out, exp_cnt = oracle.multilevel(Rf, Rc, below)
    got = np.stack([o.cpu().numpy() for o in out], 1)
    assert_bits_equal(got, exp_out, "multi-level radiance")
    assert_bits_equal(cnt.cpu().numpy().view(np.uint32), exp_cnt, "multi-level count")
    assert not np.array_equal(exp_out, Rf.out)  # the case takes coarser cells


def test_multilevel_frame_filter_moving_average(gpu):
    """FrameFilter with a coarser level and the moving average on both levels:
    four frames, each equal to the oracle's fine and coarse frames combined."""
    wl = synth.get("hd_1080p_x3")
    w, h = 480, 270
    n = w * h * 3
    flt = pf.FrameFilter(n, 20, temporal=True, alpha_old=wl.alpha_old, fused=True, multilevel=(4, 1))
    sf = sc = None
    for frame in range(4):
        f = synth.generate(wl, frame=frame, width=w, height=h)
        f["log2_slots"] = 20
        g = to_dev(f)
        out = flt.filter(g["px"], g["py"], g["pz"], g["nx"], g["ny"], g["nz"], g["valid"], g["r"], g["g"], g["b"],
                         f["cam"], f["s"], f["seed"], with_count=True)
        torch.cuda.synchronize()
        Rf = oracle.filter_frame(_host(f), prev_state=sf, temporal=True, alpha_old=wl.alpha_old)
        Rc = oracle.filter_frame(_host(f), prev_state=sc, temporal=True, alpha_old=wl.alpha_old, level_up=1)
        exp_out, exp_cnt = oracle.multilevel(Rf, Rc, 4)
        assert_bits_equal(np.stack([o.cpu().numpy() for o in out], 1), exp_out, f"frame {frame} radiance")
        assert_bits_equal(flt.count[:n].cpu().numpy().view(np.uint32), exp_cnt, f"frame {frame} count")
        sf, sc = Rf.state, Rc.state
