"""FrameFilter's staging choices give the same frames bit for bit: the
clear done in the lookup's launch and the temporal blend done in the insert
(the defaults) against a clear launch and a temporal pass of their own,
alone and with the optional stages that follow the blend; the default
staging also equals the oracle over eight frames."""
import numpy as np
import pytest
import torch

import oracle
import paper_1902_05942_amd as pf
import synth
from gpu_util import assert_bits_equal, to_dev

pytestmark = pytest.mark.gpu

W, H, LOG2 = 400, 230, 19


def _host(f):
    return {k: (v.cpu() if torch.is_tensor(v) else v) for k, v in f.items()}


def _run(flt, g, f):
    out = flt.filter(g["px"], g["py"], g["pz"], g["nx"], g["ny"], g["nz"], g["valid"], g["r"], g["g"], g["b"],
                     f["cam"], f["s"], f["seed"], with_count=True)
    torch.cuda.synchronize()
    n = g["px"].numel()
    return np.stack([o.cpu().numpy() for o in out], 1), flt.count[:n].cpu().numpy().view(np.uint32).copy()


@pytest.mark.parametrize("name,opts", [
    ("moving_average", {}),
    ("integration", {"max_samples": 40}),
    ("low_density", {"low_density": (4, pf.LD_NEIGHBOURS)}),
    ("history", {"history": (20, 8)}),
    ("multilevel", {"multilevel": (4, 1)}),
])
def test_staging_choices_agree(gpu, name, opts):
    wl = synth.get("hd_1080p_x3")
    n = W * H * 3
    common = dict(temporal=True, alpha_old=wl.alpha_old, fused=True, **opts)
    a = pf.FrameFilter(n, LOG2, **common)
    b = pf.FrameFilter(n, LOG2, clear_in_lookup=False, temporal_in_insert=False, **common)
    assert b.temporal_in_insert is False
    assert a.temporal_in_insert == (name in ("moving_average", "integration", "low_density"))
    for frame in range(8):
        f = synth.generate(wl, frame=frame, width=W, height=H)
        f["log2_slots"] = LOG2
        g = to_dev(f)
        print(f"[frame filter] {name} frame {frame}", flush=True)
        oa, ca = _run(a, g, f)
        ob, cb = _run(b, g, f)
        assert_bits_equal(oa, ob, f"{name} frame {frame} radiance")
        assert_bits_equal(ca, cb, f"{name} frame {frame} count")


@pytest.mark.parametrize("max_samples", [None, 40])
def test_default_staging_equals_the_oracle(gpu, max_samples):
    wl = synth.get("hd_1080p_x3")
    n = W * H * 3
    flt = pf.FrameFilter(n, LOG2, temporal=True, alpha_old=wl.alpha_old, fused=True, max_samples=max_samples)
    state = None
    for frame in range(8):
        f = synth.generate(wl, frame=frame, width=W, height=H)
        f["log2_slots"] = LOG2
        print(f"[frame filter] oracle max_samples={max_samples} frame {frame}", flush=True)
        out, cnt = _run(flt, to_dev(f), f)
        R = oracle.filter_frame(_host(f), prev_state=state, temporal=True, alpha_old=wl.alpha_old,
                                max_samples=max_samples)
        assert_bits_equal(out, R.out, f"frame {frame} radiance")
        assert_bits_equal(cnt, R.cnt, f"frame {frame} count")
        state = R.state
