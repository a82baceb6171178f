"""Hashed path space filtering on MI355X (gfx950).

The filter runs in libpf.so (HIP kernels behind the C ABI of include/pf.h);
this package only binds it (paper_1902_05942_amd._lib) and sequences its
calls for one frame (FrameFilter).  Importing fails loudly when libpf.so has
not been built: there is no fallback path.
"""
from __future__ import annotations

import torch

from . import _lib
from ._lib import (SLOT_BYTES, STAT_DISP, STAT_HIST, STAT_OVERFLOW, STAT_TEMPORAL_HIT, STAT_USED, SUMS_FIXED64,  # noqa
                   SUMS_FLOAT32, V_INVALID, V_KEYRANGE,
                   V_OVERFLOW, V_RADRANGE, Mlp, PfError, Table, build_keys, clear, geometry, insert_accumulate,
                   mlp_features, mlp_infer, mlp_init, mlp_select, mlp_select_workspace_bytes, mlp_train_step,
                   query_average, read_stats, table_init, temporal_update, version, table_bytes, make_view,
                   filter_views, views_workspace_bytes, filter_views_concurrent, views_concurrent_workspace_bytes, insert_workspace_bytes, insert_accumulate_binned,
                   microbench, MB_COPY, MB_GATHER, MB_SCATTER, MB_RMW, MB_CAS, temporal_integrate, MAX_SAMPLES,
                   build_keys_insert_binned, low_density_fallback, LD_NEIGHBOURS, LD_NORMALS, coarsen_keys,
                   query_multilevel, History, temporal_history, resolve_pixels, TEMPORAL_ACROSS_LEVELS,
                   query_average_clear, build_keys_insert_binned_temporal,
                   build_keys_insert_binned_noalloc, NOALLOC_SCRATCH_BYTES, NOALLOC_BATCH)


class MlpFallback:
    """Online-trained network for vertices in sparse cells: per frame, list
    the vertices of well-populated cells (count >= train_from) and of sparse
    cells (count < sparse_below), run `steps` training steps of `batch`
    samples, then replace the sparse vertices' output by the prediction."""

    def __init__(self, n_max: int, weights, batch: int = 16384, steps: int = 4, lr: float = 1e-3,
                 sparse_below: int = 4, train_from: int = 16, device="cuda"):
        self.net = Mlp(batch, device)
        mlp_init(self.net, weights)
        self.batch, self.steps, self.lr = batch, steps, lr
        self.sparse_below, self.train_from = sparse_below, train_from
        self.train_idx = torch.empty(max(n_max, 1), dtype=torch.int32, device=device)
        self.sparse_idx = torch.empty(max(n_max, 1), dtype=torch.int32, device=device)
        self.counts = torch.zeros(2, dtype=torch.int32, device=device)
        self.ws = torch.empty(max(mlp_select_workspace_bytes(n_max), 4), dtype=torch.uint8, device=device)

    def apply(self, table, geo, vflags, count, slot, out, seed, timing=None):
        """timing: optional 4 events recorded on the current stream before
        selection, after selection, after the training steps, after inference."""
        n = vflags.numel()
        if timing:
            timing[0].record()
        mlp_select(vflags, count, self.sparse_below, self.train_from, self.train_idx[:n], self.sparse_idx[:n],
                   self.counts, self.ws)
        if timing:
            timing[1].record()
        for k in range(self.steps):
            mlp_train_step(self.net, table, geo, slot, self.train_idx[:n], self.counts, self.batch,
                           (int(seed) ^ ((k + 1) * 0x9E3779B97F4A7C15)) & 0xFFFFFFFFFFFFFFFF, self.lr)
        if timing:
            timing[2].record()
        mlp_infer(self.net, geo, self.sparse_idx[:n], self.counts, out[0], out[1], out[2])
        if timing:
            timing[3].record()


class FrameFilter:
    """Per-view state across frames: two tables (current and previous) and
    the per-vertex key, flag and slot buffers.

    filter() runs one frame: clear the current table, build keys, insert,
    temporal blend against the previous frame's table, the low-density
    fallback when asked for, look up, then swap the tables.  Every step is
    one library call on the current stream.  With two tables and the plain
    lookup, clear_in_lookup empties the previous frame's table (read for the
    last time by the temporal blend) in the lookup's launch
    (pf_query_average_clear), so the next frame starts without a clear.
    With keys built in the binned insert, the moving average or integration
    against the previous frame's table, and no history, coarser level or
    search across levels, temporal_in_insert blends each cell where the
    insert finalises it (pf_build_keys_insert_binned_temporal) instead of in
    a pass of its own.
    """

    def __init__(self, n_max: int, log2_slots: int, max_probe: int = 64, frac_bits: int = 24,
                 temporal: bool = True, alpha_old: float = 0.2, agg_width: int = 0, device="cuda",
                 mlp: "MlpFallback | None" = None, binned: bool = False, float_sums: bool = False,
                 max_samples: "int | None" = None, fused: bool = False, low_density=None, multilevel=None,
                 history=None, across_levels: bool = False, clear_in_lookup: bool = True,
                 temporal_in_insert: bool = True):
        fmt = SUMS_FLOAT32 if float_sums else SUMS_FIXED64
        self.tables = [Table(log2_slots, max_probe, frac_bits, True, device, sum_format=fmt)
                       for _ in range(2 if temporal else 1)]
        for t in self.tables:
            table_init(t)
        self.log2_slots = log2_slots
        self.temporal = temporal
        self.alpha_old = alpha_old
        self.max_samples = max_samples  # None: moving average; else temporal integration with this threshold
        # (below, mode): cells with fewer vertices take the pooled value of low_density_fallback
        self.low_density = low_density
        # (log2_slots, max_age): the temporal pass blends against a History kept across frames
        self.history = History(history[0], history[1], device) if history is not None else None
        # the moving average looks for a cell whose level changed one level coarser and finer
        self.across_levels = across_levels
        if across_levels and max_samples is not None:
            raise ValueError("across_levels goes with the moving average here (pf_temporal_update mode 1 | "
                             "TEMPORAL_ACROSS_LEVELS integrates without a sample threshold)")
        # (below, levels): vertices whose cell holds fewer vertices take the cell `levels` levels coarser,
        # accumulated in a second pair of tables (multi-level accumulation)
        self.multilevel = multilevel
        self.coarse = None
        if multilevel is not None:
            self.coarse = [Table(log2_slots, max_probe, frac_bits, True, device, sum_format=fmt)
                           for _ in range(2 if temporal else 1)]
            for t in self.coarse:
                table_init(t)
            self.key_c = torch.empty(n_max, dtype=torch.int64, device=device)
            self.vflags_c = torch.empty(n_max, dtype=torch.uint8, device=device)
            self.slot_c = torch.empty(n_max, dtype=torch.int32, device=device)
        self.agg_width = agg_width
        self.key = torch.empty(n_max, dtype=torch.int64, device=device)
        self.vflags = torch.empty(n_max, dtype=torch.uint8, device=device)
        self.slot = torch.empty(n_max, dtype=torch.int32, device=device)
        self.count = torch.empty(n_max, dtype=torch.int32, device=device)
        self.frames = 0
        self.clear_in_lookup = clear_in_lookup
        self.temporal_in_insert = (temporal_in_insert and fused and temporal and history is None
                                   and multilevel is None and not across_levels)
        self._cur_clean = False  # the current table was emptied by the last frame's lookup
        self.mlp = mlp
        self.ws = None
        self.fused = fused  # keys built inside the binned insert (implies binned)
        if binned or fused:
            nb = insert_workspace_bytes(n_max, log2_slots)
            if nb == 0:
                raise PfError("pf_insert_workspace_bytes", _lib.PF_ERANGE)
            self.ws = torch.empty(nb, dtype=torch.uint8, device=device)

    @property
    def cur(self) -> Table:
        return self.tables[0]

    @property
    def prev(self):
        return self.tables[1] if (self.temporal and self.frames > 0) else None

    def filter(self, px, py, pz, nx, ny, nz, valid, r, g, b, cam, s, seed, out=None, idx_base=0,
               with_count=False, mlp_timing=None):
        """Filters one frame; returns (r_out, g_out, b_out) (in place if out is (r, g, b)).
        mlp_timing: optional 4 events for the learned fallback's stages (MlpFallback.apply)."""
        n = px.numel()
        key, vflags, slot = self.key[:n], self.vflags[:n], self.slot[:n]
        cnt = self.count[:n] if (with_count or self.mlp is not None) else None
        cur = self.cur
        if not self._cur_clean:
            clear(cur)
        self._cur_clean = False
        if self.fused:  # the keys are only written when the learned fallback or the coarser level reads them
            want_key = self.mlp is not None or self.multilevel is not None
            if self.temporal_in_insert:  # the current table is empty here (cleared, or by the last lookup)
                build_keys_insert_binned_temporal(cur, px, py, pz, nx, ny, nz, valid, cam, s, seed, idx_base, r, g,
                                                  b, key if want_key else None, vflags, slot, self.ws, self.prev,
                                                  self.alpha_old, self.max_samples or 0)
            else:
                build_keys_insert_binned(cur, px, py, pz, nx, ny, nz, valid, cam, s, seed, idx_base, r, g, b,
                                         key if want_key else None, vflags, slot, self.ws)
        else:
            build_keys(px, py, pz, nx, ny, nz, valid, cam, s, seed, idx_base, self.log2_slots, key, None, None, vflags)
            if self.ws is not None:
                insert_accumulate_binned(cur, key, r, g, b, vflags, slot, self.ws)
            else:
                insert_accumulate(cur, key, r, g, b, vflags, slot, self.agg_width)
        use_blend = self.temporal or self.low_density is not None
        levels = [] if self.temporal_in_insert else [(cur, self.prev)]
        if self.multilevel is not None:
            cc = self.coarse[0]
            key_c, vflags_c, slot_c = self.key_c[:n], self.vflags_c[:n], self.slot_c[:n]
            clear(cc)
            coarsen_keys(key, vflags, self.multilevel[1], key_c, vflags_c)
            if self.ws is not None:
                insert_accumulate_binned(cc, key_c, r, g, b, vflags_c, slot_c, self.ws)
            else:
                insert_accumulate(cc, key_c, r, g, b, vflags_c, slot_c, self.agg_width)
            levels.append((cc, self.coarse[1] if (self.temporal and self.frames > 0) else None))
        if self.history is not None and self.temporal:
            temporal_history(cur, self.history, self.alpha_old, 0 if self.max_samples is None else 1,
                             self.max_samples or MAX_SAMPLES, self.frames)
            levels = levels[1:]
        if use_blend:
            for t_cur, t_prev in levels:
                if self.max_samples is None:
                    temporal_update(t_cur, t_prev, self.alpha_old,
                                    TEMPORAL_ACROSS_LEVELS if self.across_levels else 0)
                else:
                    temporal_integrate(t_cur, t_prev, self.max_samples)
        if self.low_density is not None:
            low_density_fallback(cur, *self.low_density)
        if out is None:
            out = (torch.empty_like(r), torch.empty_like(g), torch.empty_like(b))
        if self.multilevel is not None:
            query_multilevel(cur, self.coarse[0], slot, slot_c, r, g, b, vflags, vflags_c, self.multilevel[0],
                             use_blend, out[0], out[1], out[2], cnt)
        elif self.temporal and self.clear_in_lookup:
            # the other table becomes the current one after the swap below
            query_average_clear(cur, key, slot, r, g, b, vflags, use_blend, out[0], out[1], out[2],
                                self.tables[1], cnt)
            self._cur_clean = True
        else:
            query_average(cur, key, slot, r, g, b, vflags, use_blend, out[0], out[1], out[2], cnt)
        if self.mlp is not None:
            geo = geometry(key, px, py, pz, nx, ny, nz, cam)
            self.mlp.apply(cur, geo, vflags, cnt, slot, out, seed, timing=mlp_timing)
        if self.temporal:
            self.tables.reverse()
            if self.coarse is not None:
                self.coarse.reverse()
        self.frames += 1
        return out


class MultiViewFilter:
    """Many views filtered per frame, by one persistent launch
    (mode "persistent", pf_filter_views) or by every view's single-view calls
    spread over library streams (mode "concurrent",
    pf_filter_views_concurrent); the same results.

    Each view has two tables (current, previous) carved from ONE arena, and
    its own key/flag/slot/count/output buffers.  filter() takes one frame dict
    per view (device streams px..nz, valid, r, g, b and cam, s, seed), runs
    the frame (persistent: with the given workgroup size and aggregation
    width), then swaps every view's tables.
    """

    def __init__(self, views, max_probe: int = 64, frac_bits: int = 24, temporal: bool = True,
                 alpha_old: float = 0.2, device="cuda", keys: bool = True, mode: str = "persistent"):
        # views: list of (n_max, log2_slots); keys: write every vertex's key (8 bytes a vertex)
        self.temporal, self.alpha_old, self.keys = temporal, alpha_old, keys
        sizes = [table_bytes(l, True) for _, l in views]
        ntab = 2 if temporal else 1
        total = sum(sizes) * ntab
        self.arena = torch.empty(total, dtype=torch.uint8, device=device)
        self.tables, off = [], 0
        for (n, l), sz in zip(views, sizes):
            pair = []
            for _ in range(ntab):
                pair.append(Table(l, max_probe, frac_bits, True, device, arena=self.arena[off:off + sz]))
                table_init(pair[-1])
                off += sz
            self.tables.append(pair)
        self.bufs = []
        for n, _ in views:
            self.bufs.append({
                "key": torch.empty(n, dtype=torch.int64, device=device),
                "vflags": torch.empty(n, dtype=torch.uint8, device=device),
                "slot": torch.empty(n, dtype=torch.int32, device=device),
                "count": torch.empty(n, dtype=torch.int32, device=device),
                "out": tuple(torch.empty(n, dtype=torch.float32, device=device) for _ in range(3)),
            })
        if mode not in ("persistent", "concurrent"):
            raise ValueError(f"mode {mode!r}")
        self.mode = mode
        ns, ls = [n for n, _ in views], [l for _, l in views]
        ws = views_workspace_bytes(ns, ls) if mode == "persistent" else views_concurrent_workspace_bytes(ns, ls)
        self.workspace = torch.empty(ws + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        self.ws = self.workspace[(-base) % 256:][:ws]
        self.frames = 0

    def descriptors(self, frames, with_count=False):
        descs = []
        for v, f in enumerate(frames):
            b = self.bufs[v]
            n = f["px"].numel()
            pair = self.tables[v]
            prev = pair[1] if (self.temporal and self.frames > 0) else None
            descs.append(make_view(f, b["key"][:n] if self.keys else None, b["vflags"][:n], b["slot"][:n],
                                   tuple(o[:n] for o in b["out"]), pair[0], prev,
                                   b["count"][:n] if with_count else None, self.temporal, self.alpha_old))
        return descs

    def filter(self, frames, block=256, agg_width=None, with_count=False, grid_per_cu=0, nstreams=1):
        """agg_width: None = 2 x block (windows of 2 x block vertices merged in LDS)."""
        if self.mode == "concurrent":
            filter_views_concurrent(self.descriptors(frames, with_count), self.ws, nstreams)
        else:
            agg = 2 * block if agg_width is None else agg_width
            filter_views(self.descriptors(frames, with_count), block, agg, self.ws, grid_per_cu)
        if self.temporal:
            for pair in self.tables:
                pair.reverse()
        self.frames += 1
        return [tuple(o[:f["px"].numel()] for o in b["out"]) for b, f in zip(self.bufs, frames)]

    def status(self) -> int:
        return int(self.ws[:4].view(torch.int32).cpu()[0])

    def phase_us(self):
        """Microseconds of the last launch's phases as seen by workgroup 0:
        clear, keys + insert, reduce with the temporal values, lookup."""
        w = self.ws[:64].view(torch.int32).cpu().numpy().view("uint32").astype("uint64")
        t = [int(w[4 + 2 * k]) | (int(w[5 + 2 * k]) << 32) for k in range(5)]
        hz = int(_lib.lib.pf_wall_clock_hz()) or 100_000_000
        return [(t[k + 1] - t[k]) * 1e6 / hz for k in range(4)]

    def status_words(self):
        """status, grid size, arrivals seen by a timed-out wait, its barrier number."""
        return [int(x) for x in self.ws[:16].view(torch.int32).cpu()]
