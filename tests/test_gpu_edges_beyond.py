"""Edge cases of the entry points beyond the hot path, on the GPU against the
oracle: a 16-slot table whose probe runs wrap from the last slot to the first
(low-density fallbacks, both modes, and the temporal blend done in the insert
with the lookup that empties the other table), a 16-slot history fought over for four
frames, and empty or single-vertex inputs of the multi-level calls and the
pixel resolve."""
import numpy as np
import pytest
import torch

import oracle
import paper_1902_05942_amd as pf
import synth
from gpu_util import assert_bits_equal, check_frame_against_oracle, gpu_frame, table_contents, to_dev

pytestmark = pytest.mark.gpu


def _small_cloud(max_cells=14):
    """A seeded cloud of a few vertices whose voxels fit a 16-slot table."""
    for seed in range(100):
        f = synth.mixed_normals_frame(12, seed, 0.4, spread=0.3, log2_slots=4)
        f["max_probe"] = 16
        R = oracle.filter_frame(f, temporal=False)
        if len(R.gkey) <= max_cells and R.table.order_free:
            return f, R
    raise AssertionError("no small cloud found")


@pytest.mark.parametrize("mode", [pf.LD_NEIGHBOURS, pf.LD_NORMALS])
def test_low_density_in_a_16_slot_table(gpu, mode):
    f, _ = _small_cloud()
    t = pf.Table(4, max_probe=16)
    pf.table_init(t)
    res = gpu_frame(f, to_dev(f), t, agg=64, low_density=(1 << 20, mode))
    R = oracle.filter_frame(f, temporal=False, low_density_fallback=(1 << 20, mode))
    check_frame_against_oracle(res, R, t)
    tc = table_contents(t)
    order = np.argsort(tc["key"])
    assert_bits_equal(tc["blend"][order][:, :3], R.gval[R.table.gslot >= 0], "pooled values")


def test_history_of_16_slots(gpu):
    H = pf.History(4, 2)
    Ho = oracle.History.empty(4, 2)
    t = pf.Table(10)
    pf.table_init(t)
    for k in range(4):
        f = synth.mixed_normals_frame(300, 40 + k % 2, 0.2, log2_slots=10)
        g = to_dev(f)
        n = len(f["px"])
        key = torch.empty(n, dtype=torch.int64, device="cuda")
        vflags = torch.empty(n, dtype=torch.uint8, device="cuda")
        slot = torch.empty(n, dtype=torch.int32, device="cuda")
        ws = torch.empty(pf.insert_workspace_bytes(n, 10), dtype=torch.uint8, device="cuda")
        pf.clear(t)
        pf.build_keys_insert_binned(t, g["px"], g["py"], g["pz"], g["nx"], g["ny"], g["nz"], g["valid"], f["cam"],
                                    f["s"], f["seed"], 0, g["r"], g["g"], g["b"], None, vflags, slot, ws)
        pf.temporal_history(t, H, 0.2, 0, pf.MAX_SAMPLES, k)
        out = tuple(torch.empty_like(g["r"]) for _ in range(3))
        pf.query_average(t, None, slot, g["r"], g["g"], g["b"], vflags, True, out[0], out[1], out[2], None)
        torch.cuda.synchronize()
        R = oracle.filter_frame(f, temporal=True, alpha_old=0.2, history=Ho, frame=k)
        assert_bits_equal(np.stack([o.cpu().numpy() for o in out], 1), R.out, f"frame {k} radiance")
        word = H.arrays()[0].cpu().numpy().view(np.uint64)
        assert_bits_equal(word, Ho.word, f"frame {k} history words")
        assert Ho.occupied().sum() <= 16


def test_multilevel_and_resolve_empty_and_single(gpu):
    e64 = torch.empty(0, dtype=torch.int64, device="cuda")
    e8 = torch.empty(0, dtype=torch.uint8, device="cuda")
    pf.coarsen_keys(e64, e8, 1, e64, e8)
    t = pf.Table(8)
    pf.table_init(t)
    e = torch.empty(0, device="cuda")
    ei = torch.empty(0, dtype=torch.int32, device="cuda")
    pf.query_multilevel(t, t, ei, ei, e, e, e, e8, e8, 4, False, e, e, e, None)
    # one vertex: its coarse key is its key's halved coordinates one level up
    k = torch.tensor([(7 + 65536) | ((-3 + 65536) << 17) | ((4 + 65536) << 34) | ((2 + 16) << 51) | (1 << 56)],
                     dtype=torch.int64, device="cuda")
    fl = torch.zeros(1, dtype=torch.uint8, device="cuda")
    kc = torch.empty_like(k)
    flc = torch.empty_like(fl)
    pf.coarsen_keys(k, fl, 1, kc, flc)
    torch.cuda.synchronize()
    exp = (3 + 65536) | ((-2 + 65536) << 17) | ((2 + 65536) << 34) | ((3 + 16) << 51) | (1 << 56)
    assert int(kc.cpu()[0]) == exp and int(flc.cpu()[0]) == 0
    # a level beyond the key's range
    k15 = torch.tensor([(15 + 16) << 51], dtype=torch.int64, device="cuda")
    pf.coarsen_keys(k15, fl, 1, kc, flc)
    torch.cuda.synchronize()
    assert int(flc.cpu()[0]) == pf.V_KEYRANGE and int(kc.cpu()[0]) == 0
    # resolve with no vertices per path: the image is kept (accumulate) or zeroed
    img = tuple(torch.full((5,), 2.5, device="cuda") for _ in range(3))
    one = torch.ones(5, device="cuda")
    pf.resolve_pixels(one, one, one, None, None, 5, 0, img, accumulate=True)
    torch.cuda.synchronize()
    assert all(bool((x == 2.5).all()) for x in img)
    pf.resolve_pixels(one, one, one, None, None, 5, 0, img, accumulate=False)
    torch.cuda.synchronize()
    assert all(bool((x == 0.0).all()) for x in img)


def test_temporal_in_the_insert_and_lookup_clear_in_16_slot_tables(gpu):
    """The fused insert with the temporal blend, and the lookup that empties
    the other table, on two 16-slot tables whose probe runs wrap: four frames
    (clouds A, A, B, A) against the oracle, frame 1 finding every key of
    frame 0 in the previous table."""
    clouds = []
    for seed in range(200):
        f = synth.mixed_normals_frame(12, seed, 0.4, spread=0.3, log2_slots=4)
        f["max_probe"] = 16
        R = oracle.filter_frame(f, temporal=False)
        if len(R.gkey) <= 14 and R.table.order_free:
            clouds.append(f)
        if len(clouds) == 2:
            break
    assert len(clouds) == 2
    tabs = [pf.Table(4, max_probe=16), pf.Table(4, max_probe=16)]
    for t in tabs:
        pf.table_init(t)
    state = None
    for frame, which in enumerate((0, 0, 1, 0)):
        f = clouds[which]
        cur, other = tabs[frame % 2], tabs[(frame + 1) % 2]
        print(f"[16-slot temporal in insert] frame {frame} cloud {which}", flush=True)
        res = gpu_frame(f, to_dev(f), cur, prev=other if frame else None, agg="fused", temporal=True, alpha=0.2,
                        clear=False, clear_in_lookup=other, temporal_in_insert=True)
        R = oracle.filter_frame(f, prev_state=state, temporal=True, alpha_old=0.2)
        check_frame_against_oracle(res, R, cur)
        if frame == 1:
            assert int(res["stats"][pf.STAT_TEMPORAL_HIT]) == len(R.gkey) > 0
        assert int(other.occupancy().abs().sum()) == 0
        state = R.state


def test_temporal_in_the_insert_with_no_vertices(gpu):
    """n == 0: nothing is launched and the table keeps its contents."""
    f, _ = _small_cloud()
    t, p = pf.Table(4, max_probe=16), pf.Table(4, max_probe=16)
    pf.table_init(t); pf.table_init(p)
    gpu_frame(f, to_dev(f), t, agg=64)
    before = t.arena.clone()
    e = torch.empty(0, device="cuda")
    ws = torch.empty(256, dtype=torch.uint8, device="cuda")
    pf.build_keys_insert_binned_temporal(t, e, e, e, e, e, e, None, f["cam"], f["s"], f["seed"], 0, e, e, e, None,
                                         torch.empty(0, dtype=torch.uint8, device="cuda"),
                                         torch.empty(0, dtype=torch.int32, device="cuda"), ws, p, 0.2)
    torch.cuda.synchronize()
    assert torch.equal(t.arena, before)
