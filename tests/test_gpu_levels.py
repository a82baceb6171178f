"""GPU parity of the temporal pass across levels (pf_temporal_update with
PF_TEMPORAL_ACROSS_LEVELS, Section 3.4.2) against the CPU oracle, bit for
bit, over frames of the orbit in which some voxels change level: the moving
average through FrameFilter, and integration through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
import paper_1902_05942_amd as pf
import synth
from gpu_util import assert_bits_equal, check_frame_against_oracle, gpu_frame, table_contents, to_dev

pytestmark = pytest.mark.gpu


def _host(f):
    return {k: (v.cpu() if torch.is_tensor(v) else v) for k, v in f.items()}


def test_across_levels_moving_average_frame_filter(gpu):
    wl = synth.get("hd_1080p_x3")
    w, h = 480, 270
    n = w * h * 3
    flt = pf.FrameFilter(n, 20, temporal=True, alpha_old=wl.alpha_old, fused=True, across_levels=True)
    state, changed = None, 0
    for frame in range(6):
        f = synth.generate(wl, frame=frame, width=w, height=h)
        f["log2_slots"] = 20
        g = to_dev(f)
        print(f"[levels] frame {frame}", flush=True)
        out = flt.filter(g["px"], g["py"], g["pz"], g["nx"], g["ny"], g["nz"], g["valid"], g["r"], g["g"], g["b"],
                         f["cam"], f["s"], f["seed"], with_count=True)
        torch.cuda.synchronize()
        R = oracle.filter_frame(_host(f), prev_state=state, temporal=True, alpha_old=wl.alpha_old,
                                across_levels=True)
        assert_bits_equal(np.stack([o.cpu().numpy() for o in out], 1), R.out, f"frame {frame} radiance")
        assert_bits_equal(flt.count[:n].cpu().numpy().view(np.uint32), R.cnt, f"frame {frame} count")
        if state is not None:
            plain = oracle.temporal_ema(R.gkey, R.gavg, state[0], state[1], wl.alpha_old)
            changed += int((~np.all(plain == R.gval, 1)).sum())
        state = R.state
    assert changed > 100  # voxels that found their region one level up or down


def test_across_levels_integration(gpu):
    wl = synth.get("hd_1080p_x3")
    tabs = [pf.Table(20), pf.Table(20)]
    for t in tabs:
        pf.table_init(t)
    state = None
    for frame in range(4):
        f = synth.generate(wl, frame=frame, width=320, height=180)
        f["log2_slots"] = 20
        cur, prev = tabs[frame % 2], (tabs[(frame + 1) % 2] if frame else None)
        g = to_dev(f)
        res = gpu_frame(f, g, cur, prev=None, agg="fused", temporal=False)
        pf.temporal_update(cur, prev, 0.0, 1 | pf.TEMPORAL_ACROSS_LEVELS)
        torch.cuda.synchronize()
        R = oracle.filter_frame(_host(f), prev_state=state, temporal=True, max_samples=1 << 24, across_levels=True)
        tc = table_contents(cur)
        order = np.argsort(tc["key"])
        placed = R.table.gslot >= 0
        assert_bits_equal(tc["blend"][order][:, :3], R.gval[placed], f"frame {frame} values")
        assert_bits_equal(tc["blend"][order][:, 3].astype(np.uint32), R.state[2], f"frame {frame} counts")
        state = R.state
