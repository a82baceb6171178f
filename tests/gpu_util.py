"""Helpers for the GPU parity tests: run frames through the C ABI and read
back every per-vertex and per-table result as numpy arrays."""
from __future__ import annotations

import numpy as np
import torch

import paper_1902_05942_amd as pf

FIELDS = ("px", "py", "pz", "nx", "ny", "nz", "r", "g", "b", "valid")


def to_dev(f, dev="cuda"):
    return {k: (f[k].to(dev) if torch.is_tensor(f[k]) else torch.from_numpy(np.ascontiguousarray(f[k])).to(dev))
            for k in FIELDS}


def table_contents(t: pf.Table):
    """Occupied bitmap and (key, count, sums, blend) of every occupied slot."""
    cells = t.cells()
    fp = cells[:, 0].cpu().numpy().view(np.uint32)
    occ = fp != 0
    c64 = cells.view(torch.int64)
    cnt = cells[:, 1].cpu().numpy().view(np.uint32)
    sums = c64[:, 1:4].cpu().numpy()
    keys = t.keys().cpu().numpy().view(np.uint64)
    out = {"occupied": occ.astype(np.uint8), "fp": fp[occ], "key": keys[occ], "count": cnt[occ],
           "sum": sums[occ], "slots": np.nonzero(occ)[0]}
    if t.with_blend:
        out["blend"] = t.blend().cpu().numpy()[occ]
    return out


def gpu_frame(f, g, cur: pf.Table, prev=None, agg=0, use_slot=True, temporal=False, alpha=0.2,
              idx_base=0, in_place=False, clear=True, want_fp_home=True, max_samples=None, low_density=None,
              clear_in_lookup=None, temporal_in_insert=False):
    """One frame through the C ABI; returns per-vertex results and stats.
    clear_in_lookup: a table that the lookup's launch empties
    (pf_query_average_clear) instead of the plain lookup.
    temporal_in_insert (with agg == "fused" and temporal): the temporal pass
    inside the insert (pf_build_keys_insert_binned_temporal)."""
    n = g["px"].numel()
    dev = g["px"].device
    key = torch.empty(n, dtype=torch.int64, device=dev)
    fp = torch.empty(n, dtype=torch.int32, device=dev) if want_fp_home else None
    home = torch.empty(n, dtype=torch.int32, device=dev) if want_fp_home else None
    vflags = torch.empty(n, dtype=torch.uint8, device=dev)
    slot = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.empty(n, dtype=torch.int32, device=dev)
    if clear:
        pf.clear(cur)
    if agg == "fused":
        fp = home = None
        want_fp_home = False
        ws = torch.empty(pf.insert_workspace_bytes(n, cur.log2_slots), dtype=torch.uint8, device=dev)
        if temporal_in_insert:
            pf.build_keys_insert_binned_temporal(cur, g["px"], g["py"], g["pz"], g["nx"], g["ny"], g["nz"], g["valid"],
                                                 f["cam"], f["s"], f["seed"], idx_base, g["r"], g["g"], g["b"], key,
                                                 vflags, slot, ws, prev, alpha, max_samples or 0)
        else:
            pf.build_keys_insert_binned(cur, g["px"], g["py"], g["pz"], g["nx"], g["ny"], g["nz"], g["valid"],
                                        f["cam"], f["s"], f["seed"], idx_base, g["r"], g["g"], g["b"], key, vflags,
                                        slot, ws)
        flags_keys = None
    else:
        pf.build_keys(g["px"], g["py"], g["pz"], g["nx"], g["ny"], g["nz"], g["valid"], f["cam"], f["s"], f["seed"],
                      idx_base, cur.log2_slots, key, fp, home, vflags)
        flags_keys = vflags.clone()
    if agg == "fused":
        pass
    elif agg == "binned":
        ws = torch.empty(pf.insert_workspace_bytes(n, cur.log2_slots), dtype=torch.uint8, device=dev)
        pf.insert_accumulate_binned(cur, key, g["r"], g["g"], g["b"], vflags, slot, ws)
    else:
        pf.insert_accumulate(cur, key, g["r"], g["g"], g["b"], vflags, slot if use_slot else None, agg)
    if temporal_in_insert:
        assert agg == "fused" and temporal
    elif temporal and max_samples is not None:
        pf.temporal_integrate(cur, prev, max_samples)
    elif temporal or low_density is not None:
        pf.temporal_update(cur, prev if temporal else None, alpha)
    if low_density is not None:
        pf.low_density_fallback(cur, *low_density)
        temporal = True  # the lookup returns the temporal value
    if in_place:
        out = (g["r"].clone(), g["g"].clone(), g["b"].clone())
        src = out
    else:
        out = (torch.empty_like(g["r"]), torch.empty_like(g["g"]), torch.empty_like(g["b"]))
        src = (g["r"], g["g"], g["b"])
    if clear_in_lookup is not None:
        pf.query_average_clear(cur, key, slot if use_slot else None, src[0], src[1], src[2], vflags, temporal,
                               out[0], out[1], out[2], clear_in_lookup, cnt)
    else:
        pf.query_average(cur, key, slot if use_slot else None, src[0], src[1], src[2], vflags, temporal,
                         out[0], out[1], out[2], cnt)
    torch.cuda.synchronize()
    res = {
        "key": key.cpu().numpy().view(np.uint64),
        "flags_keys": None if flags_keys is None else flags_keys.cpu().numpy(),
        "flags": vflags.cpu().numpy(),
        "out": np.stack([o.cpu().numpy() for o in out], 1),
        "cnt": cnt.cpu().numpy().view(np.uint32),
        "slot": slot.cpu().numpy().view(np.uint32),
        "stats": pf.read_stats(cur),
    }
    if want_fp_home:
        res["fp"] = fp.cpu().numpy().view(np.uint32)
        res["home"] = home.cpu().numpy().view(np.uint32)
    return res


def assert_bits_equal(a, b, what):
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    assert a.shape == b.shape, f"{what}: shape {a.shape} vs {b.shape}"
    if a.dtype.kind == "f":
        a = a.view(np.uint32 if a.dtype.itemsize == 4 else np.uint64)
        b = b.view(a.dtype)
    bad = np.nonzero(a.reshape(a.shape[0], -1) != b.reshape(b.shape[0], -1))[0] if a.ndim else []
    assert len(bad) == 0, f"{what}: {len(bad)} of {a.shape[0]} differ, first at {bad[:5]}"


def check_frame_against_oracle(res, R, t: pf.Table, table_exact=True):
    """Every per-vertex output and the order-free table facts, bit for bit."""
    assert_bits_equal(res["key"], R.key, "key")
    if "fp" in res:
        assert_bits_equal(res["fp"], R.fp, "fingerprint")
        assert_bits_equal(res["home"], R.home, "home")
    assert_bits_equal(res["flags"], R.flags, "flags")
    assert_bits_equal(res["cnt"], R.cnt, "count")
    assert_bits_equal(res["out"], R.out, "filtered radiance")
    st = res["stats"]
    G_placed = int((R.table.gslot >= 0).sum())
    assert int(st[pf.STAT_USED]) == G_placed
    assert int(st[pf.STAT_OVERFLOW]) == int(((R.flags & pf.V_OVERFLOW) != 0).sum())
    tc = table_contents(t)
    # the table as a multiset {(key, count, sums)} equals the oracle's groups
    order = np.argsort(tc["key"])
    placed = R.table.gslot >= 0
    assert_bits_equal(tc["key"][order], R.gkey[placed], "table keys")
    assert_bits_equal(tc["count"][order], R.gcnt[placed], "table counts")
    assert_bits_equal(tc["sum"][order], R.gsum[placed], "table sums")
    assert_bits_equal(tc["fp"][order], R.gfp[placed], "table fingerprints")
    if table_exact:
        assert R.table.order_free
        assert_bits_equal(tc["occupied"], R.table.occupied, "occupied slots")
        assert int(st[pf.STAT_DISP]) == R.table.total_disp
    # which key lands at which displacement depends on arrival order; the
    # histogram must still count every placed key, and its first moment must
    # be the (order-free) total displacement when no key reaches bin 64
    hist = st[pf.STAT_HIST:pf.STAT_HIST + 65].astype(np.int64)
    assert int(hist.sum()) == G_placed
    if hist[64] == 0:
        assert int((hist[:64] * np.arange(64)).sum()) == int(st[pf.STAT_DISP])
    assert int(np.nonzero(hist)[0].max(initial=0)) < max(R.table.lmax, 1)
