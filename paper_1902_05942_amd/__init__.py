"""Hashed path space filtering on MI355X (gfx950).

The filter runs in libpf.so (HIP kernels behind the C ABI of include/pf.h);
this package only binds it (paper_1902_05942_amd._lib) and sequences its
calls for one frame (FrameFilter).  Importing fails loudly when libpf.so has
not been built: there is no fallback path.
"""
from __future__ import annotations

import torch

from . import _lib
from ._lib import (STAT_DISP, STAT_HIST, STAT_OVERFLOW, STAT_TEMPORAL_HIT, STAT_USED, V_INVALID, V_KEYRANGE,  # noqa
                   V_OVERFLOW, V_RADRANGE, PfError, Table, build_keys, clear, insert_accumulate, query_average,
                   read_stats, table_init, temporal_update, version)


class FrameFilter:
    """Per-view state across frames: two tables (current and previous) and
    the per-vertex key, flag and slot buffers.

    filter() runs one frame: clear the current table, build keys, insert,
    temporal blend against the previous frame's table, look up, then swap
    the tables.  Every step is one library call on the current stream.
    """

    def __init__(self, n_max: int, log2_slots: int, max_probe: int = 64, frac_bits: int = 24,
                 temporal: bool = True, alpha_old: float = 0.2, agg_width: int = 0, device="cuda"):
        self.tables = [Table(log2_slots, max_probe, frac_bits, True, device) for _ in range(2 if temporal else 1)]
        for t in self.tables:
            table_init(t)
        self.log2_slots = log2_slots
        self.temporal = temporal
        self.alpha_old = alpha_old
        self.agg_width = agg_width
        self.key = torch.empty(n_max, dtype=torch.int64, device=device)
        self.vflags = torch.empty(n_max, dtype=torch.uint8, device=device)
        self.slot = torch.empty(n_max, dtype=torch.int32, device=device)
        self.count = torch.empty(n_max, dtype=torch.int32, device=device)
        self.frames = 0

    @property
    def cur(self) -> Table:
        return self.tables[0]

    @property
    def prev(self):
        return self.tables[1] if (self.temporal and self.frames > 0) else None

    def filter(self, px, py, pz, nx, ny, nz, valid, r, g, b, cam, s, seed, out=None, idx_base=0,
               with_count=False):
        """Filters one frame; returns (r_out, g_out, b_out) (in place if out is (r, g, b))."""
        n = px.numel()
        key, vflags, slot = self.key[:n], self.vflags[:n], self.slot[:n]
        cnt = self.count[:n] if with_count else None
        cur = self.cur
        clear(cur)
        build_keys(px, py, pz, nx, ny, nz, valid, cam, s, seed, idx_base, self.log2_slots, key, None, None, vflags)
        insert_accumulate(cur, key, r, g, b, vflags, slot, self.agg_width)
        if self.temporal:
            temporal_update(cur, self.prev, self.alpha_old)
        if out is None:
            out = (torch.empty_like(r), torch.empty_like(g), torch.empty_like(b))
        query_average(cur, key, slot, r, g, b, vflags, self.temporal, out[0], out[1], out[2], cnt)
        if self.temporal:
            self.tables.reverse()
        self.frames += 1
        return out
