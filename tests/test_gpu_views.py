"""GPU parity of the persistent multi-view launch: every view of every frame
equals the oracle bit for bit, for every (workgroup size, aggregation width)
the autotuner can pick, and on one full-size frame of the 8-view workload."""
import functools

import numpy as np
import pytest
import torch

import oracle
import paper_1902_05942_amd as pf
import synth
from paper_1902_05942_amd import autotune
from gpu_util import assert_bits_equal, table_contents

pytestmark = pytest.mark.gpu

SHAPES = [(160, 90, 3, 16), (64, 64, 1, 14), (301, 167, 3, 18), (97, 55, 2, 15)]


def _views(frame):
    wl = synth.get("multiview_8")
    out = []
    for v, (w, h, vpp, m) in enumerate(SHAPES):
        spec = synth.ViewSpec(w, h, vpp, m, synth.workloads.CONFIG_SEED + v)
        wl_v = synth.Workload(f"view{v}", [spec], frames=3)
        f = synth.generate(wl_v, frame=frame)
        f["s"] = 0.01 if v != 3 else 0.03
        out.append(f)
    return wl, out


@functools.lru_cache(maxsize=None)
def _oracle_frames():
    """The oracle's results of the three frames of every view (they do not
    depend on the launch configuration)."""
    states = [None] * len(SHAPES)
    res = []
    for frame in range(3):
        wl, fs = _views(frame)
        row = []
        for v, f in enumerate(fs):
            R = oracle.filter_frame(f, prev_state=states[v], temporal=True, alpha_old=0.2)
            row.append((R, states[v]))
            states[v] = R.state
        res.append(row)
    return res


def test_every_tuner_pick_is_tested():
    assert len(autotune.candidates()) == 25
    assert set(autotune.candidates()) == set(PICKS)


PICKS = autotune.candidates()


@pytest.mark.parametrize("block,agg", PICKS)
def test_views_bit_exact_over_frames(gpu, block, agg):
    _views_over_frames("persistent", block, agg)


def test_views_concurrent_bit_exact_over_frames(gpu):
    """The single-view calls of every view on the library's streams."""
    _views_over_frames("concurrent", 0, 0)


def _views_over_frames(mode, block, agg):
    mvf = pf.MultiViewFilter([(w * h * vpp, m) for w, h, vpp, m in SHAPES], temporal=True, alpha_old=0.2, mode=mode)
    states = [None] * len(SHAPES)
    expected = _oracle_frames()
    for frame in range(3):
        wl, fs = _views(frame)
        dev = [{k: (v.cuda() if torch.is_tensor(v) else v) for k, v in f.items()} for f in fs]
        outs = mvf.filter(dev, block, agg, with_count=True)
        torch.cuda.synchronize()
        if mode == "persistent":
            assert mvf.status() == 0, mvf.status_words()
        for v, f in enumerate(fs):
            R, _ = expected[frame][v]
            b = mvf.bufs[v]
            n = f["px"].numel()
            assert_bits_equal(b["key"][:n].cpu().numpy().view(np.uint64), R.key, f"view {v} keys")
            assert_bits_equal(b["vflags"][:n].cpu().numpy(), R.flags, f"view {v} flags")
            assert_bits_equal(b["count"][:n].cpu().numpy().view(np.uint32), R.cnt, f"view {v} counts")
            got = np.stack([o.cpu().numpy() for o in outs[v]], 1)
            assert_bits_equal(got, R.out, f"view {v} frame {frame} radiance")
            t = mvf.tables[v][1]            # this frame's table after the swap
            tc = table_contents(t)
            order = np.argsort(tc["key"])
            assert R.table.order_free
            assert_bits_equal(tc["key"][order], R.gkey, f"view {v} table keys")
            assert_bits_equal(tc["sum"][order], R.gsum, f"view {v} table sums")
            assert_bits_equal(tc["occupied"], R.table.occupied, f"view {v} occupancy")
            st = pf.read_stats(t)
            assert int(st[pf.STAT_USED]) == len(R.gkey) and int(st[pf.STAT_DISP]) == R.table.total_disp
            if frame:
                assert int(st[pf.STAT_TEMPORAL_HIT]) == int(np.isin(R.gkey, states[v][0]).sum())
            states[v] = R.state


def test_views_argument_checks(gpu):
    mvf = pf.MultiViewFilter([(100, 10)], temporal=True)
    wl, fs = _views(0)
    f = {k: (v.cuda() if torch.is_tensor(v) else v) for k, v in fs[1].items()}
    n = f["px"].numel()
    mvf2 = pf.MultiViewFilter([(n, 14)], temporal=True)
    d = mvf2.descriptors([f])
    with pytest.raises(pf.PfError):
        pf.filter_views(d, 96, 0, mvf2.ws)                 # unsupported workgroup size
    with pytest.raises(pf.PfError):
        pf.filter_views(d, 256, 768, mvf2.ws)              # aggregation width not a power of two
    with pytest.raises(pf.PfError):
        pf.filter_views(d, 256, 128, mvf2.ws)              # aggregation width below the workgroup
    with pytest.raises(pf.PfError):
        pf.filter_views(d, 256, 4096, mvf2.ws)             # aggregation width above 8 x workgroup
    with pytest.raises(pf.PfError):
        pf.filter_views(d + d, 256, 0, mvf2.ws)            # two views sharing tables
    d[0].r_out = d[0].r
    with pytest.raises(pf.PfError):
        pf.filter_views(d, 256, 0, mvf2.ws)                # output aliasing the input
    del mvf


def test_views_concurrent_argument_checks(gpu):
    wl, fs = _views(0)
    f = {k: (v.cuda() if torch.is_tensor(v) else v) for k, v in fs[1].items()}
    n = f["px"].numel()
    mvf = pf.MultiViewFilter([(n, 14)], temporal=True, mode="concurrent")
    d = mvf.descriptors([f])
    for ns in (0, 5):
        with pytest.raises(pf.PfError):
            pf.filter_views_concurrent(d, mvf.ws, nstreams=ns)          # stream count outside 1..4
    with pytest.raises(pf.PfError):
        pf.filter_views_concurrent(d, mvf.ws[:1024], nstreams=1)        # workspace too small
    with pytest.raises(pf.PfError):
        pf.filter_views_concurrent(d + d, mvf.ws, nstreams=2)           # two views sharing tables
    d[0].r_out = d[0].r
    with pytest.raises(pf.PfError):
        pf.filter_views_concurrent(d, mvf.ws, nstreams=1)               # output aliasing the input


def test_eight_views_full_size_one_frame(gpu):
    """One frame of the full 8-view workload (59.5M vertex slots, per-view
    tables of 2^19 .. 2^24 slots in one arena) at the configuration the
    benchmark's tuner picked most often, every view against the oracle."""
    wl = synth.get("multiview_8")
    shapes = [(v.width * v.height * v.verts_per_path, v.log2_slots) for v in wl.views]
    mvf = pf.MultiViewFilter(shapes, wl.max_probe, wl.frac_bits, temporal=True, alpha_old=wl.alpha_old)
    for frame in range(2):
        fs = [synth.generate(wl, view=v, frame=frame) for v in range(len(wl.views))]
        print(f"multiview_8 frame {frame}: {sum(f['px'].numel() for f in fs)} slots", flush=True)
        dev = [{k: (x.cuda() if torch.is_tensor(x) else x) for k, x in f.items()} for f in fs]
        outs = mvf.filter(dev, 256, 512, with_count=True)
        torch.cuda.synchronize()
        assert mvf.status() == 0
        if frame == 0:
            states = []
            for v, f in enumerate(fs):
                states.append(oracle.filter_frame(f, temporal=True, alpha_old=wl.alpha_old).state)
            continue
        for v, f in enumerate(fs):
            R = oracle.filter_frame(f, prev_state=states[v], temporal=True, alpha_old=wl.alpha_old)
            b = mvf.bufs[v]
            n = f["px"].numel()
            assert_bits_equal(b["key"][:n].cpu().numpy().view(np.uint64), R.key, f"view {v} keys")
            assert_bits_equal(b["vflags"][:n].cpu().numpy(), R.flags, f"view {v} flags")
            assert_bits_equal(b["count"][:n].cpu().numpy().view(np.uint32), R.cnt, f"view {v} counts")
            got = np.stack([o.cpu().numpy() for o in outs[v]], 1)
            assert_bits_equal(got, R.out, f"view {v} radiance")
            t = mvf.tables[v][1]
            tc = table_contents(t)
            order = np.argsort(tc["key"])
            assert R.table.order_free
            assert_bits_equal(tc["key"][order], R.gkey, f"view {v} table keys")
            assert_bits_equal(tc["count"][order], R.gcnt, f"view {v} table counts")
            assert_bits_equal(tc["sum"][order], R.gsum, f"view {v} table sums")
            assert_bits_equal(tc["occupied"], R.table.occupied, f"view {v} occupancy")
            st = pf.read_stats(t)
            assert int(st[pf.STAT_USED]) == len(R.gkey) and int(st[pf.STAT_DISP]) == R.table.total_disp
            assert int(st[pf.STAT_TEMPORAL_HIT]) == int(np.isin(R.gkey, states[v][0]).sum())


def test_eight_views_full_size_concurrent_equals_persistent(gpu):
    """Two frames of the full 8-view workload through the single-view calls
    on the library's streams and through the persistent launch (checked
    against the oracle above): every output, flag and count equal, and every
    table's cells (by key) and occupied slots (linear probing occupies the
    same slots in any order of insertion; which of two colliding keys takes
    the first depends on the order)."""
    wl = synth.get("multiview_8")
    shapes = [(v.width * v.height * v.verts_per_path, v.log2_slots) for v in wl.views]
    filters = [pf.MultiViewFilter(shapes, wl.max_probe, wl.frac_bits, temporal=True, alpha_old=wl.alpha_old,
                                  keys=False, mode=m) for m in ("persistent", "concurrent")]
    for frame in range(2):
        fs = [synth.generate(wl, view=v, frame=frame) for v in range(len(wl.views))]
        dev = [{k: (x.cuda() if torch.is_tensor(x) else x) for k, x in f.items()} for f in fs]
        outs = [mvf.filter(dev, 1024, 4096, with_count=True) for mvf in filters]
        torch.cuda.synchronize()
        assert filters[0].status() == 0
        for v in range(len(fs)):
            for a, b in zip(outs[0][v], outs[1][v]):
                assert torch.equal(a.view(torch.int32), b.view(torch.int32)), (frame, v)
            for name in ("vflags", "count"):  # slots: which of two colliding keys sits first depends on order
                n = fs[v]["px"].numel()
                assert torch.equal(filters[0].bufs[v][name][:n], filters[1].bufs[v][name][:n]), (frame, v, name)
            ta, tb = (table_contents(mvf.tables[v][1]) for mvf in filters)
            oa, ob = np.argsort(ta["key"]), np.argsort(tb["key"])
            for k in ("key", "count", "sum", "blend"):
                assert np.array_equal(ta[k][oa], tb[k][ob]), (frame, v, k)
            assert np.array_equal(ta["occupied"], tb["occupied"]), (frame, v)
        del dev


def test_views_without_temporal_blend_concurrent_equals_persistent(gpu):
    """Views filtered without the moving average (the plain lookup, no
    previous table): both ways of filtering many views give the same
    outputs, flags and counts over two frames."""
    filters = [pf.MultiViewFilter([(w * h * vpp, m) for w, h, vpp, m in SHAPES], temporal=False, mode=m)
               for m in ("persistent", "concurrent")]
    for frame in range(2):
        wl, fs = _views(frame)
        dev = [{k: (v.cuda() if torch.is_tensor(v) else v) for k, v in f.items()} for f in fs]
        outs = [mvf.filter(dev, 256, 512, with_count=True) for mvf in filters]
        torch.cuda.synchronize()
        assert filters[0].status() == 0
        for v, f in enumerate(fs):
            n = f["px"].numel()
            for a, b in zip(outs[0][v], outs[1][v]):
                assert torch.equal(a.view(torch.int32), b.view(torch.int32)), (frame, v)
            for name in ("vflags", "count"):
                assert torch.equal(filters[0].bufs[v][name][:n], filters[1].bufs[v][name][:n]), (frame, v, name)
