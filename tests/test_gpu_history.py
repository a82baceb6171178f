"""GPU parity of the history with eviction by priority (pf_history_*,
pf_temporal_history) against the CPU oracle, bit for bit: every frame's
output, the temporal-hit count, and the whole history (words, keys, values,
stamps of its occupied slots), which the single atomic minimum per slot makes
independent of the order of arrival.  Cases: the moving average over an
orbit, temporal integration, a revisited view found again after a frame
away, and a small history where most voxels collide and are evicted."""
import numpy as np
import pytest
import torch

import oracle
import paper_1902_05942_amd as pf
import synth
from gpu_util import assert_bits_equal, to_dev

pytestmark = pytest.mark.gpu


def _host(f):
    return {k: (v.cpu() if torch.is_tensor(v) else v) for k, v in f.items()}


def _run(frames, log2_hist, max_age, mode=0, max_samples=pf.MAX_SAMPLES, alpha=0.2, log2_slots=20):
    t = pf.Table(log2_slots)
    pf.table_init(t)
    H = pf.History(log2_hist, max_age)
    Ho = oracle.History.empty(log2_hist, max_age)
    for k, f in enumerate(frames):
        f["log2_slots"] = log2_slots
        g = to_dev(f)
        n = g["px"].numel()
        print(f"[history] frame {k} n={n} log2_hist={log2_hist} max_age={max_age} mode={mode}", flush=True)
        key = torch.empty(n, dtype=torch.int64, device="cuda")
        vflags = torch.empty(n, dtype=torch.uint8, device="cuda")
        slot = torch.empty(n, dtype=torch.int32, device="cuda")
        cnt = torch.empty(n, dtype=torch.int32, device="cuda")
        ws = torch.empty(pf.insert_workspace_bytes(n, log2_slots), dtype=torch.uint8, device="cuda")
        pf.clear(t)
        pf.build_keys_insert_binned(t, g["px"], g["py"], g["pz"], g["nx"], g["ny"], g["nz"], g["valid"], f["cam"],
                                    f["s"], f["seed"], 0, g["r"], g["g"], g["b"], None, vflags, slot, ws)
        pf.temporal_history(t, H, alpha, mode, max_samples, k)
        out = tuple(torch.empty_like(g["r"]) for _ in range(3))
        pf.query_average(t, None, slot, g["r"], g["g"], g["b"], vflags, True, out[0], out[1], out[2], cnt)
        torch.cuda.synchronize()
        R = oracle.filter_frame(_host(f), temporal=True, alpha_old=alpha, history=Ho, frame=k,
                                max_samples=None if mode == 0 else max_samples)
        assert R.table.order_free
        assert_bits_equal(np.stack([o.cpu().numpy() for o in out], 1), R.out, f"frame {k} radiance")
        assert_bits_equal(cnt.cpu().numpy().view(np.uint32), R.cnt, f"frame {k} count")
        word, hkey, hval, stamp = (a.cpu().numpy() for a in H.arrays())
        word = word.view(np.uint64)
        assert_bits_equal(word, Ho.word, f"frame {k} history words")
        occ = Ho.occupied()
        assert_bits_equal(hkey.view(np.uint64)[occ], Ho.key[occ], f"frame {k} history keys")
        assert_bits_equal(hval[occ], Ho.val[occ], f"frame {k} history values")
        assert_bits_equal(stamp.view(np.uint32)[occ], Ho.stamp[occ], f"frame {k} history stamps")
        hits = int(pf.read_stats(t)[pf.STAT_TEMPORAL_HIT])
        yield k, R, Ho, hits


def _orbit(n, w=480, h=270, start=0):
    wl = synth.get("hd_1080p_x3")
    return [synth.generate(wl, frame=start + k, width=w, height=h) for k in range(n)]


def test_history_moving_average_orbit(gpu):
    seen = 0
    for k, R, Ho, hits in _run(_orbit(6), 20, 3):
        seen += hits
    assert seen > 1000


def test_history_integration(gpu):
    for k, R, Ho, hits in _run(_orbit(4, 320, 180), 20, 2, mode=1, max_samples=16):
        pass
    assert int(Ho.val[Ho.occupied(), 3].max()) == 16  # the sample threshold binds


def test_history_finds_a_revisited_view(gpu):
    a, b = _orbit(1, 320, 180)[0], _orbit(1, 320, 180, start=12)[0]
    frames = [a, b, synth.generate(synth.get("hd_1080p_x3"), frame=0, width=320, height=180)]
    res = list(_run(frames, 21, 4))
    k, R, Ho, hits = res[2]
    # frame 2 repeats frame 0 (same view and jitter): nearly all its voxels
    # are found again, more than frame 1 found from frame 0
    assert hits > 0.8 * (R.table.gslot >= 0).sum()
    assert hits > res[1][3]


def test_history_small_table_evicts_by_priority(gpu):
    for k, R, Ho, hits in _run(_orbit(5, 320, 180), 12, 2):
        # 4096 slots for ~20k voxels a frame: every slot is fought over
        assert Ho.occupied().sum() > 3500
