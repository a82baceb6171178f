"""GPU parity of the low-density fallbacks (pf_low_density_fallback) against
the CPU oracle, bit for bit: the small scene at two voxel sizes, a cloud of
mixed normals where the probe-run search pools many voxels, a scaled frame
with a ragged tail, the full 1080p x3 frame in the benchmark's launch
configuration, and a run of frames with the moving average."""
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


def _check_values(t, R):
    """The temporal value of every placed cell equals the oracle's (pooled
    where the fallback applied, the cell's own average elsewhere)."""
    tc = table_contents(t)
    order = np.argsort(tc["key"])
    placed = R.table.gslot >= 0
    assert_bits_equal(tc["blend"][order][:, :3], R.gval[placed], "cell values")


def _case(case):
    if case.startswith("tiny"):
        f = synth.generate(synth.get("tiny_64x64"))
        f["s"] = float(case.split("_")[1])
        return f, 0
    if case == "mixed":
        return synth.mixed_normals_frame(3000, 11, 0.08), 0
    if case == "scaled_ragged":
        return synth.generate(synth.get("hd_1080p_x3"), frame=2, width=401, height=229), "binned"
    return synth.generate(synth.get("hd_1080p_x3"), frame=0, device="cuda"), "fused"


@pytest.mark.parametrize("mode", [pf.LD_NEIGHBOURS, pf.LD_NORMALS])
@pytest.mark.parametrize("case,below", [("tiny_0.01", 4), ("tiny_0.1", 64), ("mixed", 6), ("scaled_ragged", 4),
                                        ("hd_full", 4)])
def test_low_density_bit_exact(gpu, case, below, mode):
    f, agg = _case(case)
    print(f"[low_density] {case} below={below} mode={mode} n={len(f['px'])}", flush=True)
    g = to_dev(f)
    t = pf.Table(f["log2_slots"], f["max_probe"], f["frac_bits"])
    pf.table_init(t)
    res = gpu_frame(f, g, t, agg=agg, low_density=(below, mode))
    R = oracle.filter_frame(_host(f), temporal=False, low_density_fallback=(below, mode))
    check_frame_against_oracle(res, R, t)
    _check_values(t, R)
    if mode == pf.LD_NEIGHBOURS or case == "mixed":
        # the case exercises the fallback (the scenes' axis-aligned faces put
        # one normal class per position, so only the cloud pools normals)
        P = oracle.filter_frame(_host(f), temporal=False)
        assert not np.array_equal(R.out, P.out)


def test_low_density_threshold_one_changes_nothing(gpu):
    f, _ = _case("tiny_0.01")
    g = to_dev(f)
    t = pf.Table(f["log2_slots"], f["max_probe"], f["frac_bits"])
    pf.table_init(t)
    for mode in (pf.LD_NEIGHBOURS, pf.LD_NORMALS):
        res = gpu_frame(f, g, t, agg=64, low_density=(1, mode))
        check_frame_against_oracle(res, oracle.filter_frame(_host(f), temporal=False), t)


@pytest.mark.parametrize("mode", [pf.LD_NEIGHBOURS, pf.LD_NORMALS])
def test_low_density_with_moving_average_frames(gpu, mode):
    """Six frames of the orbit with the moving average and the fallback: the
    pooled values enter the next frame's blend as its previous values."""
    wl = synth.get("hd_1080p_x3")
    tabs = [pf.Table(20), pf.Table(20)]
    for t in tabs:
        pf.table_init(t)
    state = None
    for frame in range(6):
        f = synth.generate(wl, frame=frame, width=480, height=270)
        f["log2_slots"] = 20
        cur, prev = tabs[frame % 2], (tabs[(frame + 1) % 2] if frame else None)
        res = gpu_frame(f, to_dev(f), cur, prev=prev, agg="fused", temporal=True, alpha=wl.alpha_old,
                        low_density=(4, mode))
        R = oracle.filter_frame(_host(f), prev_state=state, temporal=True, alpha_old=wl.alpha_old,
                                low_density_fallback=(4, mode))
        check_frame_against_oracle(res, R, cur)
        _check_values(cur, R)
        state = R.state


def test_frame_filter_with_low_density(gpu):
    """The package's FrameFilter (fused insert) runs the fallback between the
    temporal pass and the lookup."""
    wl = synth.get("hd_1080p_x3")
    f = synth.generate(wl, frame=5, width=640, height=360)
    f["log2_slots"] = 20
    g = to_dev(f)
    n = g["px"].numel()
    flt = pf.FrameFilter(n, 20, temporal=False, fused=True, low_density=(4, pf.LD_NEIGHBOURS))
    out = flt.filter(g["px"], g["py"], g["pz"], g["nx"], g["ny"], g["nz"], g["valid"], g["r"], g["g"], g["b"],
                     f["cam"], f["s"], f["seed"], with_count=True)
    torch.cuda.synchronize()
    R = oracle.filter_frame(_host(f), temporal=False, low_density_fallback=(4, pf.LD_NEIGHBOURS))
    assert_bits_equal(np.stack([o.cpu().numpy() for o in out], 1), R.out, "filtered radiance")
    assert_bits_equal(flt.count[:n].cpu().numpy().view(np.uint32), R.cnt, "count")
