"""Benchmark: hashed path space filtering of the 1080p x3 workload on one GPU.

One step filters one frame of the orbiting camera (1920x1080 pixels, 3 path
vertex slots per pixel, 6,220,800 vertex slots): build keys and
insert-accumulate into the current table with the temporal moving average
against the previous frame's table done where the insert finalises each
cell (--separate-temporal: a temporal pass of its own), then look up,
emptying the previous frame's table in the lookup's launch for the next
frame (--separate-clear: a clear launch at the start of each frame).
Sixteen frames are generated on the GPU before timing (inputs resident in
HBM) and steps cycle through them.

Prints one JSON line.  `value` is vertices filtered per second (valid
vertices, i.e. those with a hit, over the whole timed region); per-kernel
times come from HIP events on the stream the kernels run on.

Other workloads (--workload):
  hd_1080p_x3_mlp  the same frames with the learned fallback for sparse
                   cells (4 training steps of 16384 samples and inference
                   per frame); reports RMSE with and without it.
  multiview_8      8 views of uneven resolution (59.5M vertex slots) in one
                   persistent launch per frame, workgroup size and
                   aggregation width chosen by the autotuner.
  uhd_4k_x4        3840x2160x4 (33.2M slots, 2^25-slot table): a real frame,
                   then synthetic key streams at table loads 0.1-0.7 for
                   probe limits 32, 64, 128 (insert + lookup per point,
                   displacement statistics, overflow counts).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=160)
    p.add_argument("--warmup", type=int, default=16)
    p.add_argument("--workload", default="hd_1080p_x3")
    p.add_argument("--agg", type=int, default=64, help="aggregation width of insert (0 = none)")
    p.add_argument("--insert", choices=("atomic", "binned", "fused"), default="fused",
                   help="binned: vertices merged per chunk in LDS, one record per group, reduced per slot range "
                        "without atomics on the sums; fused: the same with the keys built inside it; atomic: device "
                        "atomics per aggregated group")
    p.add_argument("--frames", type=int, default=16)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-legs", action="store_true",
                   help="leave out the learned-fallback, 8-view and 4K blocks of the default run")
    p.add_argument("--cpu-workers", type=int, default=0,
                   help="host processes for the all-cores oracle timing (0 = the cores this process may use, at "
                        "most 16)")
    p.add_argument("--cpu-frames", type=int, default=8, help="frames of the oracle timed on the host")
    p.add_argument("--lean", action="store_true",
                   help="time the frames only (no probes, segments, quality or oracle legs): for profiler runs")
    p.add_argument("--probes", action="store_true",
                   help="with --lean: run the random-access probes after the frames (counter runs of both)")
    p.add_argument("--low-density", default="",
                   help="below,mode: add the low-density fallback (mode 0 neighbourhood, 1 similar normals) for "
                        "cells with fewer than `below` vertices, timed as its own stage")
    p.add_argument("--multilevel", default="",
                   help="below,levels: also accumulate every vertex `levels` levels coarser in a second pair of tables "
                        "and look up the coarser cell for cells with fewer than `below` vertices, timed per stage")
    p.add_argument("--history", default="",
                   help="log2_slots,max_age: blend against a history kept across frames with eviction by priority "
                        "instead of the previous frame's table")
    p.add_argument("--across-levels", action="store_true",
                   help="the temporal pass also searches a changed cell's region one level coarser and finer")
    p.add_argument("--resolve", action="store_true",
                   help="add the pixel resolve (value times the path throughput, summed per pixel) as a stage")
    p.add_argument("--separate-temporal", action="store_true",
                   help="run the temporal pass as a launch of its own instead of inside the fused insert")
    p.add_argument("--separate-clear", action="store_true",
                   help="clear each frame's table in its own launch instead of in the previous frame's lookup")
    p.add_argument("--copy-probe-mib", type=int, default=0,
                   help="only run an elementwise copy of this many MiB 4 times (calibrates HBM byte counters)")
    return p.parse_args()


def source_digest():
    """SHA-256 over the HIP sources and the C header, in name order: a traffic
    figure measured with hardware counters is reported only while it still
    describes the kernels as built."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1902_05942_amd", "csrc")
    files = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".hip", ".h")))
    for f in files + [os.path.join(ROOT, "include", "pf.h")]:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counter_profile(workload, mode):
    """Fields of the committed counter summary
    profiles/hbm_traffic_<workload>_<mode>.txt (HBM bytes per call of each
    stage from FETCH_SIZE and WRITE_SIZE, each scaled by the same counter's
    reading for a copy of known size, and the bytes fetched per random
    32-byte gather of the probe), or {} when there is none or the sources
    changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}_{mode}.txt")
    if not os.path.exists(path):
        return {}
    fields = {}
    with open(path) as fh:
        for line in fh:
            k, sep, v = line.partition(": ")
            if sep and not line.startswith("#") and k and " " not in k:
                fields[k] = v.strip()
    if fields.get("sources_sha256") != source_digest():
        return {}
    return fields


def counted_traffic(stage, workload, mode):
    """Counted HBM bytes per call of `stage`, or None (no summary, or the
    sources changed since it was taken)."""
    v = counter_profile(workload, mode).get(f"stage_bytes.{stage}")
    return None if v is None else int(float(v))


def copy_probe(mib):
    """An elementwise copy of known size (reads and writes `mib` MiB per
    launch), run alone so that a counter run can scale FETCH_SIZE and
    WRITE_SIZE to bytes."""
    import torch
    dev = torch.device("cuda:0")
    src = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(4):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": mib << 20, "copy_probe_bytes_written": mib << 20,
                      "launches": 4, "kernel": "torch elementwise mul (out of place)"}), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU (the filter has no multi-GPU path); got --gpus {a.gpus}",
              file=sys.stderr)
        sys.exit(2)
    if a.copy_probe_mib:
        return copy_probe(a.copy_probe_mib)
    if a.workload == "multiview_8":
        return main_multiview(a)
    if a.workload == "uhd_4k_x4":
        return main_uhd(a)
    import numpy as np
    import torch

    import paper_1902_05942_amd as pf
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    wl = synth.get(a.workload)
    view = wl.views[0]
    n = view.width * view.height * view.verts_per_path
    print(f"[bench] generating {a.frames} frames of {a.workload} ({n} slots) on {dev}", file=sys.stderr, flush=True)
    frames = [synth.generate(wl, frame=i, device=dev) for i in range(a.frames)]
    n_valid = [int(f["valid"].sum()) for f in frames]
    torch.cuda.synchronize()

    use_mlp = bool(wl.extra.get("mlp"))
    fb = None
    if use_mlp:
        from synth.mlp_init import init_params
        fb = pf.MlpFallback(n, init_params(1902), batch=16384, steps=4, lr=1e-3)
    flt = pf.FrameFilter(n, view.log2_slots, wl.max_probe, wl.frac_bits, temporal=True, alpha_old=wl.alpha_old,
                         agg_width=a.agg, device=dev, binned=(a.insert == "binned"), fused=(a.insert == "fused"))
    outs = (torch.empty(n, device=dev), torch.empty(n, device=dev), torch.empty(n, device=dev))
    count = torch.empty(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    fused = a.insert == "fused"
    low_density = tuple(int(x) for x in a.low_density.split(",")) if a.low_density else None
    multilevel = tuple(int(x) for x in a.multilevel.split(",")) if a.multilevel else None
    hist = pf.History(*(int(x) for x in a.history.split(","))) if a.history else None
    pixels = view.width * view.height
    image = tuple(torch.empty(pixels, device=dev) for _ in range(3))
    if multilevel:
        ctabs = [pf.Table(view.log2_slots, wl.max_probe, wl.frac_bits, True, dev) for _ in range(2)]
        for t in ctabs:
            pf.table_init(t)
        key_c = torch.empty(n, dtype=torch.int64, device=dev)
        vflags_c = torch.empty(n, dtype=torch.uint8, device=dev)
        slot_c = torch.empty(n, dtype=torch.int32, device=dev)
        ws_c = flt.ws if flt.ws is not None else torch.empty(pf.insert_workspace_bytes(n, view.log2_slots),
                                                             dtype=torch.uint8, device=dev)

    clear_in_lookup = not multilevel and not a.separate_clear
    # the temporal blend done where the fused insert finalises each cell
    temporal_in_insert = fused and not (multilevel or hist is not None or a.across_levels or a.separate_temporal)

    def stages(k):
        """(name, call) of one frame's steps, in order"""
        f = frames[k % len(frames)]
        key, vflags, slot = flt.key[:n], flt.vflags[:n], flt.slot[:n]
        cur = flt.cur
        # the plain lookup empties the other table in its launch (it was read
        # for the last time by the temporal pass), so the next frame's table
        # starts empty and no clear stage runs; the first frame's table is
        # empty from its initialisation
        st = [] if clear_in_lookup else [("clear", lambda: pf.clear(cur))]
        if temporal_in_insert:
            prev = flt.prev
            st.append(("build_keys_insert_temporal", lambda: pf.build_keys_insert_binned_temporal(
                cur, f["px"], f["py"], f["pz"], f["nx"], f["ny"], f["nz"], f["valid"], f["cam"], f["s"], f["seed"], 0,
                f["r"], f["g"], f["b"], key if use_mlp else None, vflags, slot, flt.ws, prev, wl.alpha_old)))
        elif fused:
            st.append(("build_keys_insert", lambda: pf.build_keys_insert_binned(
                cur, f["px"], f["py"], f["pz"], f["nx"], f["ny"], f["nz"], f["valid"], f["cam"], f["s"], f["seed"], 0,
                f["r"], f["g"], f["b"], key if (use_mlp or multilevel) else None, vflags, slot, flt.ws)))
        else:
            st.append(("build_keys", lambda: pf.build_keys(f["px"], f["py"], f["pz"], f["nx"], f["ny"], f["nz"],
                                                           f["valid"], f["cam"], f["s"], f["seed"], 0,
                                                           view.log2_slots, key, None, None, vflags)))
            if flt.ws is not None:
                st.append(("insert_accumulate",
                           lambda: pf.insert_accumulate_binned(cur, key, f["r"], f["g"], f["b"], vflags, slot, flt.ws)))
            else:
                st.append(("insert_accumulate",
                           lambda: pf.insert_accumulate(cur, key, f["r"], f["g"], f["b"], vflags, slot, a.agg)))
        if temporal_in_insert:
            pass
        elif hist is not None:
            fr = flt.frames
            st.append(("temporal_history", lambda: pf.temporal_history(cur, hist, wl.alpha_old, 0, pf.MAX_SAMPLES,
                                                                       fr)))
        else:
            st.append(("temporal_update", lambda: pf.temporal_update(
                cur, flt.prev, wl.alpha_old, pf.TEMPORAL_ACROSS_LEVELS if a.across_levels else 0)))
        if low_density:
            st.append(("low_density", lambda: pf.low_density_fallback(cur, *low_density)))
        if multilevel:
            cc, cp = ctabs[k % 2], (ctabs[(k + 1) % 2] if flt.frames else None)

            def coarse_level():
                pf.clear(cc)
                pf.coarsen_keys(key, vflags, multilevel[1], key_c, vflags_c)
                pf.insert_accumulate_binned(cc, key_c, f["r"], f["g"], f["b"], vflags_c, slot_c, ws_c)
                pf.temporal_update(cc, cp, wl.alpha_old)
            st.append(("coarse_level", coarse_level))
            st.append(("query_multilevel", lambda: pf.query_multilevel(
                cur, cc, slot, slot_c, f["r"], f["g"], f["b"], vflags, vflags_c, multilevel[0], True, outs[0],
                outs[1], outs[2], count if use_mlp else None)))
        elif clear_in_lookup:
            other = flt.tables[1]
            st.append(("query_average_clear", lambda: pf.query_average_clear(
                cur, key, slot, f["r"], f["g"], f["b"], vflags, True, outs[0], outs[1], outs[2], other,
                count if use_mlp else None)))
        else:
            st.append(("query_average", lambda: pf.query_average(cur, key, slot, f["r"], f["g"], f["b"], vflags, True,
                                                                 outs[0], outs[1], outs[2],
                                                                 count if use_mlp else None)))
        if a.resolve:
            st.append(("resolve_pixels", lambda: pf.resolve_pixels(outs[0], outs[1], outs[2],
                                                                   (f["tr"], f["tg"], f["tb"]), f["valid"],
                                                                   pixels, view.verts_per_path, image)))
        if use_mlp:
            def mlp():
                geo = pf.geometry(key, f["px"], f["py"], f["pz"], f["nx"], f["ny"], f["nz"], f["cam"])
                fb.apply(cur, geo, vflags, count, slot, outs, f["seed"], timing=mlp_ev["now"])
            st.append(("mlp_select_train_infer", mlp))
        return st

    names = [nm for nm, _ in stages(0)]
    mlp_ev = {"now": None, "all": []}

    def step(k, ev=None):
        if use_mlp:
            mlp_ev["now"] = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if ev is not None else None
            if ev is not None:
                mlp_ev["all"].append(mlp_ev["now"])
        for j, (nm, call) in enumerate(stages(k)):
            if ev is not None:
                ev[j].record(stream)
            call()
        if ev is not None:
            ev[len(names)].record(stream)
        flt.tables.reverse()
        flt.frames += 1

    print(f"[bench] warmup {a.warmup} steps", file=sys.stderr, flush=True)
    for k in range(a.warmup):
        step(k)
    torch.cuda.synchronize()

    nev = len(names) + 1
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(nev)] for _ in range(a.steps)]
    print(f"[bench] timing {a.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        step(a.warmup + k, events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = events[0][0].elapsed_time(events[-1][nev - 1])
    per = {nm: float(np.mean([events[k][j].elapsed_time(events[k][j + 1]) for k in range(a.steps)])) * 1e3
           for j, nm in enumerate(names)}  # microseconds
    spread = {nm: [round(float(np.percentile([events[k][j].elapsed_time(events[k][j + 1]) * 1e3
                                              for k in range(a.steps)], q)), 2) for q in (10, 50, 90)]
              for j, nm in enumerate(names)}
    # the slowest timed frame of each stage and its index (0 = first timed frame)
    slowest = {}
    for j, nm in enumerate(names):
        t = [events[k][j].elapsed_time(events[k][j + 1]) * 1e3 for k in range(a.steps)]
        slowest[nm] = [round(float(max(t)), 2), int(np.argmax(t))]
    valid_total = sum(n_valid[(a.warmup + k) % len(frames)] for k in range(a.steps))
    ms_per_step = wall * 1e3 / a.steps
    value = valid_total / wall

    # statistics of the last frame (untimed): cells, displacement, temporal hits
    st = pf.read_stats(flt.prev)
    cells = int(st[pf.STAT_USED])
    if a.lean:
        ra = random_access(dev, (1 << view.log2_slots) * pf.SLOT_BYTES) if a.probes else None
        print(json.dumps({"metric": "per-stage microseconds (lean profiling run)", "kernel_us":
                          {k: round(v, 2) for k, v in per.items()}, "ms_per_step": round(wall * 1e3 / a.steps, 4),
                          "insert": a.insert, "steps": a.steps, "random_access": ra}), flush=True)
        return

    # the random-access denominators, measured at the table's footprint right
    # after the timed frames, in the state the frames ran in
    ra = random_access(dev, (1 << view.log2_slots) * pf.SLOT_BYTES)

    # quality: RMSE against the noise-free radiance over valid vertices (evaluation only)
    def rmse(x, f):
        v = f["valid"].bool()
        est = torch.stack(x, 1)[v]
        return float(torch.sqrt(((est - f["truth"][v]) ** 2).mean()))
    f_last = frames[(a.warmup + a.steps - 1) % len(frames)]
    q_temporal = rmse(outs, f_last)
    mlp_info = None
    if use_mlp:
        sparse = (flt.vflags[:n] == 0) & (count < 4)
        q_sparse_mlp = float(torch.sqrt(((torch.stack(outs, 1)[sparse] - f_last["truth"][sparse]) ** 2).mean()))
        ref = pf.FrameFilter(n, view.log2_slots, wl.max_probe, wl.frac_bits, temporal=True, alpha_old=wl.alpha_old,
                             agg_width=a.agg, device=dev)
        for k in range(a.frames):   # the moving average alone over the same frames, ending on the same one
            fk = frames[(a.warmup + a.steps - a.frames + k) % len(frames)]
            o_ref = ref.filter(fk["px"], fk["py"], fk["pz"], fk["nx"], fk["ny"], fk["nz"], fk["valid"], fk["r"],
                               fk["g"], fk["b"], fk["cam"], fk["s"], fk["seed"])
        q_sparse_ref = float(torch.sqrt(((torch.stack(o_ref, 1)[sparse] - f_last["truth"][sparse]) ** 2).mean()))
        # the paper's own fallbacks for the same cells (Sections 3.3.1, 3.2.2, 3.3.2), over the same frames
        q_ld = {}
        for name, opt in (("neighbours", {"low_density": (4, pf.LD_NEIGHBOURS)}),
                          ("normals", {"low_density": (4, pf.LD_NORMALS)}),
                          ("multilevel_1", {"multilevel": (4, 1)})):
            ldf = pf.FrameFilter(n, view.log2_slots, wl.max_probe, wl.frac_bits, temporal=True,
                                 alpha_old=wl.alpha_old, device=dev, fused=True, **opt)
            for k in range(a.frames):
                fk = frames[(a.warmup + a.steps - a.frames + k) % len(frames)]
                o_ld = ldf.filter(fk["px"], fk["py"], fk["pz"], fk["nx"], fk["ny"], fk["nz"], fk["valid"], fk["r"],
                                  fk["g"], fk["b"], fk["cam"], fk["s"], fk["seed"])
            q_ld[name] = {"rmse_sparse": round(float(torch.sqrt(((torch.stack(o_ld, 1)[sparse] -
                                                                   f_last["truth"][sparse]) ** 2).mean())), 5),
                          "rmse_all": round(rmse(o_ld, f_last), 5)}
        mlp_us = per["mlp_select_train_infer"]
        flops = 4 * 16384 * 2 * (10240 + 15360)
        train_us = float(np.mean([e[1].elapsed_time(e[2]) for e in mlp_ev["all"]])) * 1e3
        select_us = float(np.mean([e[0].elapsed_time(e[1]) for e in mlp_ev["all"]])) * 1e3
        infer_us = float(np.mean([e[2].elapsed_time(e[3]) for e in mlp_ev["all"]])) * 1e3
        mlp_info = {"sparse_vertices": int(sparse.sum()), "rmse_sparse_without": round(q_sparse_ref, 5),
                    "rmse_sparse_with": round(q_sparse_mlp, 5), "rmse_all_without": round(rmse(o_ref, f_last), 5),
                    "rmse_all_with": round(q_temporal, 5), "us_per_frame": round(mlp_us, 2),
                    "select_us": round(select_us, 2), "train_us": round(train_us, 2), "infer_us": round(infer_us, 2),
                    "train_flops_per_frame": flops,
                    "train_bf16_tflops": round(flops / (train_us * 1e-6) / 1e12, 3),
                    "train_frac_of_mfma_peak": round(flops / (train_us * 1e-6) / 2.5e15, 5),
                    "loss": float(fb.net.loss().cpu()[0]),
                    "paper_fallbacks_below_4": q_ld}
    q_noisy = rmse((f_last["r"], f_last["g"], f_last["b"]), f_last)
    plain = pf.FrameFilter(n, view.log2_slots, wl.max_probe, wl.frac_bits, temporal=False, agg_width=a.agg,
                           device=dev)
    o2 = plain.filter(f_last["px"], f_last["py"], f_last["pz"], f_last["nx"], f_last["ny"], f_last["nz"],
                      f_last["valid"], f_last["r"], f_last["g"], f_last["b"], f_last["cam"], f_last["s"],
                      f_last["seed"])
    q_plain = rmse(o2, f_last)

    # the image of the last frame (Section 3: each vertex's value times its
    # path throughput, summed per pixel) against the noise-free image
    def resolved(vals):
        img = tuple(torch.empty(pixels, device=dev) for _ in range(3))
        pf.resolve_pixels(*[x.contiguous() for x in vals], (f_last["tr"], f_last["tg"], f_last["tb"]),
                          f_last["valid"], pixels, view.verts_per_path, img)
        return torch.stack(img, 1)
    tr_last = f_last["truth"]
    img_truth = resolved((tr_last[:, 0], tr_last[:, 1], tr_last[:, 2]))

    def img_rmse(vals):
        return round(float(torch.sqrt(((resolved(vals) - img_truth) ** 2).mean())), 5)
    image_rmse = {"noisy": img_rmse((f_last["r"], f_last["g"], f_last["b"])), "filtered": img_rmse(o2),
                  "filtered_temporal": img_rmse(outs), "pixels": pixels,
                  "mean_pixel_truth": round(float(img_truth.mean()), 5)}

    # roofline of the dominant kernel: algorithmic bytes per launch / mean launch time
    nv = float(np.mean(n_valid))
    algo_bytes = {
        "clear": cells * 32 + (1 << view.log2_slots) // 8,
        "build_keys": n * (6 * 4 + 1 + 8 + 1),
        "insert_accumulate": n * (1 + 4) + nv * (8 + 12 + 4 + 28),
        "temporal_update": cells * (32 + 8 + 4 + 8 + 16 + 16) + (1 << view.log2_slots) // 8,
        "query_average": n * (1 + 12) + nv * (4 + 16) + (n - nv) * 12,
        "query_average_clear": n * (1 + 12) + nv * (4 + 16) + (n - nv) * 12 + cells * 32 + (1 << view.log2_slots) // 8,
        # fused: positions, normals, valid in; flags and slot out; contribution, probe, cell update per valid vertex
        "build_keys_insert": n * (6 * 4 + 1 + 1 + 4) + nv * (12 + 4 + 28),
        # the same and the temporal pass's per-cell bytes (no bitmap scan: the owner of each cell blends it)
        "build_keys_insert_temporal": n * (6 * 4 + 1 + 1 + 4) + nv * (12 + 4 + 28) + cells * (32 + 8 + 4 + 8 + 16 + 16),
    }
    dom = max((k for k in per if k in algo_bytes), key=lambda k: per[k])
    achieved = algo_bytes[dom] / (per[dom] * 1e-6) / 1e9
    launches = {"insert_accumulate": ("aggregate, colscan, scatter (bin starts scanned in it), reduce"
                                      if a.insert == "binned" else "insert"),
                "build_keys_insert": "aggregate (keys built in it), colscan, scatter (bin starts scanned in it), reduce",
                "build_keys_insert_temporal": "aggregate (keys built in it), colscan, scatter (bin starts scanned in it), "
                                              "reduce (temporal blend in it)"}
    roofline = {"bound": "hbm", "kernel": dom, "launch": launches.get(dom, dom), "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": counted_traffic(dom, a.workload, a.insert),
                "algorithmic_bytes_per_launch": int(algo_bytes[dom])}

    # random-access roofline of the headline (insert + query): per valid vertex
    # the method makes a probe and a cell update when inserting and a probe and
    # a cell read when looking up, plus one claim per cell (4V + C touches)
    touches = 4 * nv + cells
    # fused: keys counted in the insert (and the temporal pass, when it is done there)
    t_ins = (per.get("build_keys_insert", per.get("build_keys_insert_temporal")) if fused
             else per["insert_accumulate"])
    t_q = per.get("query_average", per.get("query_average_clear", per.get("query_multilevel", 0.0)))
    t_iq = (t_ins + t_q) * 1e-6   # with the fused clear, the lookup's time includes emptying the other table
    ra["insert_query_touches"] = int(touches)
    ra["achieved_G_touches_per_s"] = round(touches / t_iq / 1e9, 2)
    # achieved random-access bandwidth: the headline calls' counted HBM bytes
    # per second over the counted bytes per second of the random 32-byte
    # gather probe at the table's footprint (the same counters, the probe's
    # rate measured live); both move whole lines, so the ratio compares like
    # with like and the probe, which does nothing but random line fetches,
    # bounds it
    prof = counter_profile(a.workload, a.insert)
    ins_name = "build_keys_insert_temporal" if temporal_in_insert else ("build_keys_insert" if fused
                                                                         else "insert_accumulate")
    q_name = "query_average_clear" if clear_in_lookup else "query_average"
    b_ins, b_q = prof.get(f"stage_bytes.{ins_name}"), prof.get(f"stage_bytes.{q_name}")
    per_gather = prof.get("probe_fetch_bytes_per_gather")
    if b_ins and b_q and per_gather:
        got = (float(b_ins) + float(b_q)) / t_iq
        probe = ra["G_per_s"]["gather_32B"] * 1e9 * float(per_gather)
        ra["headline_counted_GB_per_s"] = round(got / 1e9, 1)
        ra["gather_counted_GB_per_s"] = round(probe / 1e9, 1)
        ra["frac_of_random_access_bw"] = round(got / probe, 4)
    else:
        ra["frac_of_random_access_bw"] = None

    legs = {"mlp": None, "multiview": None, "uhd_4k": None}
    if a.workload == "hd_1080p_x3" and not a.no_legs:
        # the other configurations, each as one block of this line: the learned
        # fallback on the same frames, one 8-view launch, the 4K frame
        print("[bench] learned fallback leg", file=sys.stderr, flush=True)
        legs["mlp"] = mlp_leg(frames, wl, dev)
        print("[bench] 8-view leg", file=sys.stderr, flush=True)
        legs["multiview"] = multiview_leg(a, dev, steps=20, warmup=4)
        print("[bench] 4K leg", file=sys.stderr, flush=True)
        legs["uhd_4k"] = uhd_leg(a, dev, probes=(64,), reps=10)
    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(frames, wl, a.cpu_frames, a.cpu_workers)

    line = {
        "metric": "vertices/s filtered (insert+query) at 1080p; RMSE vs noise-free mean",
        "value": round(value, 1), "unit": "vertices/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32+int64", "data": "synthetic",
        "config": {"workload": a.workload, "width": view.width, "height": view.height,
                   "verts_per_path": view.verts_per_path, "vertex_slots": n, "valid_vertices_mean": round(nv, 1),
                   "log2_slots": view.log2_slots, "max_probe": wl.max_probe, "frac_bits": wl.frac_bits,
                   "frames": a.frames, "alpha_old": wl.alpha_old, "insert": a.insert,
                   **({"agg_width": a.agg} if a.insert == "atomic" else {}),
                   "parallelism": "single-gpu"},
        "vertex_slots_per_s": round(n * a.steps / wall, 1),
        "gpu_ms_per_step": round(gpu_ms / a.steps, 4),
        "insert_query_vertices_per_s": round(nv / t_iq, 1),
        "kernel_us": {k: round(v, 2) for k, v in per.items()},
        "kernel_us_p10_p50_p90": spread,
        "kernel_us_max_at_frame": slowest,
        "segments": segments(dev, frames[(a.warmup + a.steps - 1) % len(frames)], view, wl),
        "cells_last_frame": cells,
        "rmse": {"unfiltered": round(q_noisy, 5), "filtered": round(q_plain, 5), "filtered_temporal": round(q_temporal, 5)},
        "image_rmse": image_rmse,
        "mlp": mlp_info or legs["mlp"],
        "multiview": legs["multiview"],
        "uhd_4k": legs["uhd_4k"],
        "roofline": roofline,
        "random_access": ra,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def main_multiview(a):
    """8 views of uneven resolution in one call per frame (the faster of the
    persistent launch and the views' single-view calls on library streams)."""
    import torch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    leg = multiview_leg(a, dev, a.steps, a.warmup, verbose=True)
    line = {
        "metric": "vertices/s filtered (insert+query), 8 views in one call",
        "value": leg["vertices_per_s"], "unit": "vertices/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(leg["us_per_frame"] * 1e-3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32+int64", "data": "synthetic",
        "config": dict(leg["config"], parallelism="single-gpu"),
        **{k: v for k, v in leg.items() if k not in ("config", "vertices_per_s")},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def multiview_leg(a, dev, steps, warmup, verbose=False):
    """The 8-view workload (59.5M vertex slots, per-view tables in one arena):
    the autotuner's pick over every (workgroup, aggregation width) pair, then
    `steps` timed launches cycling over 4 frames, next to the same frames
    sent view by view through the single-view calls."""
    import numpy as np
    import torch

    import paper_1902_05942_amd as pf
    from paper_1902_05942_amd import autotune
    import synth

    wl = synth.get("multiview_8")
    nfr = min(a.frames, 4)
    shapes = [(v.width * v.height * v.verts_per_path, v.log2_slots) for v in wl.views]
    print(f"[bench] generating {nfr} frames x {len(wl.views)} views ({sum(s for s, _ in shapes)} slots)",
          file=sys.stderr, flush=True)
    frames = [[synth.generate(wl, view=v, frame=i, device=dev) for v in range(len(wl.views))] for i in range(nfr)]
    n_valid = [sum(int(f["valid"].sum()) for f in fr) for fr in frames]
    # the keys are not written (as the fused single-view insert does not write them)
    mvf = pf.MultiViewFilter(shapes, wl.max_probe, wl.frac_bits, temporal=True, alpha_old=wl.alpha_old, device=dev,
                             keys=False)
    block, agg, table = autotune.tune(mvf, frames[0], reps=3, use_cache=False, verbose=verbose)
    print(f"[bench] autotuned workgroup {block}, aggregation width {agg}", file=sys.stderr, flush=True)
    for k in range(warmup):
        mvf.filter(frames[k % nfr], block, agg)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        mvf.filter(frames[(warmup + k) % nfr], block, agg)
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert mvf.status() == 0
    phases = [round(x, 1) for x in mvf.phase_us()]
    launch_us = float(np.mean([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])) * 1e3
    valid_total = sum(n_valid[(warmup + k) % nfr] for k in range(steps))
    n_total = sum(s for s, _ in shapes)
    nv = float(np.mean(n_valid))
    cells = 0
    for pair in mvf.tables:
        cells += int(pf.read_stats(pair[1])[pf.STAT_USED])
    words = sum((1 << l) // 8 for _, l in shapes)
    # the same frames view by view through the single-view calls (fused insert, moving average), one stream:
    # what the batched launch competes with
    flts = [pf.FrameFilter(nn, l, wl.max_probe, wl.frac_bits, temporal=True, alpha_old=wl.alpha_old, device=dev,
                           fused=True) for nn, l in shapes]

    def seq_frame(fr):
        for flt, f in zip(flts, fr):
            flt.filter(f["px"], f["py"], f["pz"], f["nx"], f["ny"], f["nz"], f["valid"], f["r"], f["g"], f["b"],
                       f["cam"], f["s"], f["seed"])
    for k in range(warmup):
        seq_frame(frames[k % nfr])
    torch.cuda.synchronize()
    sev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    sev[0].record()
    for k in range(steps):
        seq_frame(frames[(warmup + k) % nfr])
    sev[1].record()
    torch.cuda.synchronize()
    seq_us = sev[0].elapsed_time(sev[1]) * 1e3 / steps
    del flts, mvf
    torch.cuda.empty_cache()
    # the same frames through pf_filter_views_concurrent: every view's single-view calls, the views spread over
    # 1..3 library streams (the tuner's pick), largest first
    mvc = pf.MultiViewFilter(shapes, wl.max_probe, wl.frac_bits, temporal=True, alpha_old=wl.alpha_old, device=dev,
                             keys=False, mode="concurrent")
    nstreams, stream_ms = autotune.tune_streams(mvc, frames[0], reps=5)
    print(f"[bench] concurrent views: {nstreams} streams", file=sys.stderr, flush=True)
    for k in range(warmup):
        mvc.filter(frames[k % nfr], nstreams=nstreams)
    torch.cuda.synchronize()
    cev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    t1 = time.perf_counter()
    cev[0].record()
    for k in range(steps):
        mvc.filter(frames[(warmup + k) % nfr], nstreams=nstreams)
    cev[1].record()
    torch.cuda.synchronize()
    conc_wall = time.perf_counter() - t1
    conc_us = cev[0].elapsed_time(cev[1]) * 1e3 / steps
    del mvc, frames
    torch.cuda.empty_cache()
    # per slot: position/normal/valid 25 read, key/flags/slot 13 written, lookup flags+slot 5 read, output 12
    # written; per valid vertex: contribution 12, probe 4, cell update 28, temporal value 16; per invalid slot:
    # own contribution 12; per cell: clear 32, temporal 84; the occupancy bitmaps read twice (the records
    # between the insert and the reduce are the implementation's, not the method's, and are not counted)
    algo = n_total * 55 + nv * 60 + (n_total - nv) * 12 + cells * 116 + 2 * words
    achieved = algo / (launch_us * 1e-6) / 1e9
    best = "concurrent" if conc_us < launch_us else "persistent"
    return {
        # the faster of the two ways the library filters many views in one call
        "mode": best, "us_per_frame": round(min(conc_us, launch_us), 2),
        "vertices_per_s": round(nv / (min(conc_us, launch_us) * 1e-6), 1),
        "config": {"workload": "multiview_8", "views": [[v.width, v.height, v.verts_per_path] for v in wl.views],
                   "vertex_slots": n_total, "valid_vertices_mean": round(nv, 1), "table_slots":
                   sum(1 << l for _, l in shapes), "block": block, "agg_width": agg, "frames": nfr,
                   "streams": nstreams},
        "concurrent": {"us_per_frame": round(conc_us, 2), "streams": nstreams,
                       "ms_per_frame_wall": round(conc_wall * 1e3 / steps, 4),
                       "tuner_ms": {str(k): round(v, 4) for k, v in sorted(stream_ms.items())}},
        "persistent_ms_per_step_wall": round(wall * 1e3 / steps, 4),
        "persistent_vertices_per_s_wall": round(valid_total / wall, 1),
        "launch_us": round(launch_us, 2),
        "launch_vertices_per_s": round(nv / (launch_us * 1e-6), 1),
        "phase_us_last_launch": {"clear": phases[0], "keys_insert": phases[1], "reduce_temporal": phases[2],
                                 "lookup": phases[3]},
        "autotune_ms": {f"{b}/{g}": round(v, 4) for (b, g), v in sorted(table.items())},
        "views_one_by_one_us": round(seq_us, 2),
        "roofline": {"bound": "hbm", "kernel": "views_kernel", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": counted_traffic("views_kernel", "multiview_8", "persistent"),
                     "algorithmic_bytes_per_launch": int(algo)},
    }


def main_uhd(a):
    """3840x2160x4 (33,177,600 slots, 2^25-slot table): a real frame at the
    default scale, then synthetic key streams at table loads 0.1 .. 0.7 for
    probe limits 32, 64, 128."""
    import torch
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    leg = uhd_leg(a, dev, probes=(32, 64, 128), reps=max(3, min(a.steps, 20)))
    line = {
        "metric": "vertices/s filtered (insert+query) at 3840x2160x4 per table load",
        "value": leg["scene"]["vertices_per_s"], "unit": "vertices/s", "n_gpus": 1, "steps": leg["reps"],
        "warmup": 1, "ms_per_step": round((leg["scene"]["insert_us"] + leg["scene"]["query_us"]) * 1e-3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32+int64", "data": "synthetic",
        "config": dict(leg["config"], parallelism="single-gpu"),
        "scene": leg["scene"], "scene_small_cells": leg["scene_small_cells"], "key_sweep": leg["key_sweep"],
    }
    print(json.dumps(line), flush=True)


def uhd_leg(a, dev, probes, reps):
    """3840x2160x4 (33,177,600 slots, 2^25-slot table): a real frame at the
    default scale (and at s / 5, more cells), then synthetic key streams at
    table loads 0.1 .. 0.7 for each probe limit in `probes`.  Per point:
    insert (binned) + lookup time, achieved load, mean displacement,
    displacement percentiles and histogram, overflow."""
    import numpy as np
    import torch

    import paper_1902_05942_amd as pf
    import synth

    wl = synth.get("uhd_4k_x4")
    m = wl.views[0].log2_slots
    n = 3840 * 2160 * 4
    key = torch.empty(n, dtype=torch.int64, device=dev)
    vflags = torch.empty(n, dtype=torch.uint8, device=dev)
    slot = torch.empty(n, dtype=torch.int32, device=dev)
    outs = [torch.empty(n, device=dev) for _ in range(3)]
    ws = torch.empty(pf.insert_workspace_bytes(n, m), dtype=torch.uint8, device=dev)

    def timed(t, keys_fn, r, g, b):
        """mean insert and lookup microseconds over reps (after one warm-up)"""
        ti, tq = [], []
        for k in range(reps + 1):
            pf.clear(t)
            keys_fn()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record()
            pf.insert_accumulate_binned(t, key, r, g, b, vflags, slot, ws)
            ev[1].record()
            pf.query_average(t, key, slot, r, g, b, vflags, False, outs[0], outs[1], outs[2], None)
            ev[2].record()
            torch.cuda.synchronize()
            if k:
                ti.append(ev[0].elapsed_time(ev[1]) * 1e3)
                tq.append(ev[1].elapsed_time(ev[2]) * 1e3)
        return float(np.mean(ti)), float(np.mean(tq))

    def point(t, nvalid, ti, tq):
        st = pf.read_stats(t)
        used = int(st[pf.STAT_USED])
        hist = st[pf.STAT_HIST:pf.STAT_HIST + 65].astype(np.int64)
        cum = np.cumsum(hist) / max(used, 1)
        return {"cells": used, "load": round(used / (1 << m), 4), "valid_vertices": nvalid,
                "insert_us": round(ti, 1), "query_us": round(tq, 1),
                "vertices_per_s": round(nvalid / ((ti + tq) * 1e-6), 1),
                "mean_displacement": round(int(st[pf.STAT_DISP]) / max(used, 1), 3),
                "displacement_p50": int(np.searchsorted(cum, 0.5)), "displacement_p99": int(np.searchsorted(cum, 0.99)),
                "displacement_max": int(np.nonzero(hist)[0].max(initial=0)), "displacement_hist_le8":
                [int(x) for x in hist[:9]], "overflow_vertices": int(st[pf.STAT_OVERFLOW])}

    print("[bench] 4K frame", file=sys.stderr, flush=True)
    f = synth.generate(wl, frame=0, device=dev)
    nvalid = int(f["valid"].sum())
    t = pf.Table(m, wl.max_probe, wl.frac_bits, with_blend=False)
    pf.table_init(t)
    frame = None
    for s in (wl.s, wl.s / 5):
        def keys_fn(s=s):
            pf.build_keys(f["px"], f["py"], f["pz"], f["nx"], f["ny"], f["nz"], f["valid"], f["cam"], s, f["seed"], 0,
                          m, key, None, None, vflags)
        ti, tq = timed(t, keys_fn, f["r"], f["g"], f["b"])
        pt = dict(point(t, nvalid, ti, tq), s=s)
        frame = frame or pt
        print(f"[bench] scene s={s}: {json.dumps(pt)}", file=sys.stderr, flush=True)
        scene_small = pt
    del f, t
    sweep = []
    for load in (0.1, 0.3, 0.5, 0.7):
        d = synth.synthetic_keys(n, int(load * (1 << m)), device=dev)
        for P in probes:
            tp = pf.Table(m, P, wl.frac_bits, with_blend=False)
            pf.table_init(tp)

            def keys_fn(d=d):
                key.copy_(d["key"])
                vflags.zero_()
            ti, tq = timed(tp, keys_fn, d["r"], d["g"], d["b"])
            pt = dict(point(tp, n, ti, tq), target_load=load, max_probe=P)
            print(f"[bench] keys load {load} P {P}: {json.dumps(pt)}", file=sys.stderr, flush=True)
            sweep.append(pt)
            del tp
        del d
    del key, vflags, slot, outs, ws
    torch.cuda.empty_cache()
    return {"reps": reps, "config": {"workload": "uhd_4k_x4", "vertex_slots": n, "log2_slots": m,
                                     "insert": "binned"},
            "scene": frame, "scene_small_cells": scene_small, "key_sweep": sweep}


def mlp_leg(frames, wl, dev):
    """The learned fallback for sparse cells on the same 1080p frames (the
    network trained online from scratch, 4 steps of 16384 samples per frame):
    16 frames to train, then 32 timed frames; RMSE against the noise-free
    radiance with and without it (and the paper's own fallbacks for the same
    cells) on the last frame, and the cost per frame."""
    import numpy as np
    import torch

    import paper_1902_05942_amd as pf
    from synth.mlp_init import init_params

    view = wl.views[0]
    n = view.width * view.height * view.verts_per_path
    warm, timed = 16, 32
    fb = pf.MlpFallback(n, init_params(1902), batch=16384, steps=4, lr=1e-3)
    flt = pf.FrameFilter(n, view.log2_slots, wl.max_probe, wl.frac_bits, temporal=True, alpha_old=wl.alpha_old,
                         device=dev, fused=True, mlp=fb)
    nfr = len(frames)

    def run(fl, k, **kw):
        f = frames[k % nfr]
        return fl.filter(f["px"], f["py"], f["pz"], f["nx"], f["ny"], f["nz"], f["valid"], f["r"], f["g"], f["b"],
                         f["cam"], f["s"], f["seed"], **kw)
    for k in range(warm):
        run(flt, k)
    torch.cuda.synchronize()
    # whole frames with the fallback, events between frames only (an event
    # recorded between two kernels costs a few microseconds of idle GPU)
    fe = [torch.cuda.Event(enable_timing=True) for _ in range(timed + 1)]
    fe[0].record()
    for k in range(warm, warm + timed):
        run(flt, k)
        fe[k - warm + 1].record()
    torch.cuda.synchronize()
    frame_with_us = float(np.mean([fe[k].elapsed_time(fe[k + 1]) for k in range(timed)])) * 1e3
    # the stages' split, from further frames with events between the stages
    split = 8
    evs = []
    t_wall = time.perf_counter()
    for k in range(warm + timed, warm + timed + split):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
        e[0].record()
        out = run(flt, k, mlp_timing=e[1:5])
        e[5].record()
        evs.append(e)
    torch.cuda.synchronize()
    wall_us = (time.perf_counter() - t_wall) * 1e6 / split
    ms = lambda i, j: float(np.mean([e[i].elapsed_time(e[j]) for e in evs])) * 1e3  # noqa: E731
    select_us, train_us, infer_us = ms(1, 2), ms(2, 3), ms(3, 4)
    last = warm + timed + split - 1
    f_last = frames[last % nfr]
    n_ = n
    sparse = (flt.vflags[:n_] == 0) & (flt.count[:n_] < 4)
    truth = f_last["truth"]
    valid = f_last["valid"].bool()

    def rmse(o, msk):
        return float(torch.sqrt(((torch.stack(o, 1)[msk] - truth[msk]) ** 2).mean()))
    q_with, q_with_all = rmse(out, sparse), rmse(out, valid)
    res = {}
    frame_without_us = None
    # the same 16 frames ending on the same one: the moving average alone (its last 12 frames timed as the
    # frames with the fallback were), then the paper's fallbacks
    for name, opt in (("without", {}), ("neighbours", {"low_density": (4, pf.LD_NEIGHBOURS)}),
                      ("normals", {"low_density": (4, pf.LD_NORMALS)}), ("multilevel_1", {"multilevel": (4, 1)})):
        ref = pf.FrameFilter(n, view.log2_slots, wl.max_probe, wl.frac_bits, temporal=True, alpha_old=wl.alpha_old,
                             device=dev, fused=True, **opt)
        we = [torch.cuda.Event(enable_timing=True) for _ in range(17)]
        for j, k in enumerate(range(last - 15, last + 1)):
            o = run(ref, k)
            we[j + 1].record()
        if name == "without":
            torch.cuda.synchronize()
            frame_without_us = float(np.mean([we[j].elapsed_time(we[j + 1]) for j in range(4, 16)])) * 1e3
        res[name] = {"rmse_sparse": round(rmse(o, sparse), 5), "rmse_all": round(rmse(o, valid), 5)}
        del ref
    flops = fb.steps * fb.batch * 2 * (10240 + 15360)
    mlp_us = frame_with_us - frame_without_us
    return {"workload": "hd_1080p_x3_mlp", "frames_trained_before_timing": warm, "timed_frames": timed,
            "sparse_vertices": int(sparse.sum()),
            "rmse_sparse_without": res["without"]["rmse_sparse"], "rmse_sparse_with": round(q_with, 5),
            "rmse_all_without": res["without"]["rmse_all"], "rmse_all_with": round(q_with_all, 5),
            # the fallback's cost: frames with it minus the same frames without it, events between frames only
            "us_per_frame": round(mlp_us, 2),
            "frame_gpu_us_without": round(frame_without_us, 2), "frame_gpu_us_with": round(frame_with_us, 2),
            "frame_wall_us_python_driven": round(wall_us, 2),
            # the stages, from frames with events between them (each such event adds a few microseconds)
            "select_us": round(select_us, 2), "train_us": round(train_us, 2), "infer_us": round(infer_us, 2),
            "train_flops_per_frame": flops, "train_bf16_tflops": round(flops / (train_us * 1e-6) / 1e12, 3),
            "train_frac_of_mfma_peak": round(flops / (train_us * 1e-6) / 2.5e15, 5),
            "loss": float(fb.net.loss().cpu()[0]),
            "paper_fallbacks_below_4": {k: v for k, v in res.items() if k != "without"}}


def segments(dev, f, view, wl, reps=20):
    """The paper separates coherent primary hits from incoherent bounces
    (Section 4): key construction + binned insert and the lookup timed on
    the primary segment (the first W*H slots) and on the bounce segments
    alone, each into a fresh table (medians of `reps` after one warm-up)."""
    import numpy as np
    import torch

    import paper_1902_05942_amd as pf
    wh = view.width * view.height
    n = f["px"].numel()
    out = {}
    for name, lo, hi in (("primary", 0, wh), ("bounces", wh, n)):
        m = hi - lo
        sl = {k: f[k][lo:hi] for k in ("px", "py", "pz", "nx", "ny", "nz", "valid", "r", "g", "b")}
        t = pf.Table(view.log2_slots, wl.max_probe, wl.frac_bits, with_blend=False, device=dev)
        pf.table_init(t)
        vflags = torch.empty(m, dtype=torch.uint8, device=dev)
        slot = torch.empty(m, dtype=torch.int32, device=dev)
        o = [torch.empty(m, device=dev) for _ in range(3)]
        ws = torch.empty(pf.insert_workspace_bytes(m, view.log2_slots), dtype=torch.uint8, device=dev)
        ti, tq = [], []
        for k in range(reps + 1):
            pf.clear(t)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record()
            pf.build_keys_insert_binned(t, sl["px"], sl["py"], sl["pz"], sl["nx"], sl["ny"], sl["nz"], sl["valid"],
                                        f["cam"], f["s"], f["seed"], lo, sl["r"], sl["g"], sl["b"], None, vflags,
                                        slot, ws)
            ev[1].record()
            pf.query_average(t, None, slot, sl["r"], sl["g"], sl["b"], vflags, False, o[0], o[1], o[2], None)
            ev[2].record()
            torch.cuda.synchronize()
            if k:
                ti.append(ev[0].elapsed_time(ev[1]) * 1e3)
                tq.append(ev[1].elapsed_time(ev[2]) * 1e3)
        nv = int(sl["valid"].sum())
        cells = int(pf.read_stats(t)[pf.STAT_USED])
        tki, tkq = float(np.median(ti)), float(np.median(tq))
        out[name] = {"slots": m, "valid_vertices": nv, "cells": cells, "build_keys_insert_us": round(tki, 1),
                     "query_us": round(tkq, 1), "vertices_per_s": round(nv / ((tki + tkq) * 1e-6), 1)}
        del t, ws
    return out


def random_access(dev, footprint):
    """Measured denominators at the table's footprint (library probe
    kernels): random 32-byte gathers, scatters, cell read-modify-writes with
    the insert's atomics and compare-and-swaps per second, and the copy
    bandwidth over 1 GiB."""
    import torch

    import paper_1902_05942_amd as pf
    buf = torch.empty(footprint, dtype=torch.uint8, device=dev)
    buf.zero_()
    rates = {}
    for name, kind in (("gather_32B", pf.MB_GATHER), ("scatter_32B", pf.MB_SCATTER), ("cell_rmw", pf.MB_RMW),
                       ("cas", pf.MB_CAS)):
        pf.microbench(kind, buf, 32, 4)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        n = sum(pf.microbench(kind, buf, 32, 8, seed=11 + r) for r in range(3))
        ev[1].record()
        torch.cuda.synchronize()
        rates[name] = round(n / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9, 2)
    del buf
    big = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    pf.microbench(pf.MB_COPY, big)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    moved = sum(2 * pf.microbench(pf.MB_COPY, big) for _ in range(3))
    ev[1].record()
    torch.cuda.synchronize()
    copy = moved / (ev[0].elapsed_time(ev[1]) * 1e-3) / 1e9
    del big
    return {"footprint_bytes": footprint, "G_per_s": rates, "copy_GB_per_s": round(copy, 1)}


def _oracle_worker(wname, frame0, k, barrier, results):
    """One host process of the all-cores timing: the oracle on frames
    frame0+1 .. frame0+k of the workload (moving average; frame0 only
    builds the previous state), timed after every process is ready."""
    import torch
    torch.set_num_threads(1)
    import oracle
    import synth
    wl = synth.get(wname)
    fr = [synth.generate(wl, frame=frame0 + i) for i in range(k + 1)]
    state = oracle.filter_frame(fr[0], temporal=True, alpha_old=wl.alpha_old).state
    barrier.wait()
    t0 = time.perf_counter()
    nv = 0
    for i in range(1, k + 1):
        state = oracle.filter_frame(fr[i], prev_state=state, temporal=True, alpha_old=wl.alpha_old).state
        nv += int(fr[i]["valid"].sum())
    results.put((t0, time.perf_counter(), nv))


def host_cores():
    """Cores this process may run on, at most 16 (the host cores that go with one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
    if env > 0:
        n = min(n, env)
    return max(1, min(n, 16))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(frames, wl, k, workers=0):
    """The oracle (single-threaded C plus numpy glue, not tuned for speed) on
    the same workload with the moving average, vertices/s over valid
    vertices: on one host thread (k consecutive frames), and on every core
    this process may use (one process per core, each filtering its own 2
    consecutive frames, all started together; the rate is all their valid
    vertices over the span from the first start to the last end)."""
    import multiprocessing as mp

    import oracle
    hosts = [{kk: (v.cpu() if hasattr(v, "cpu") else v) for kk, v in frames[i].items()} for i in range(k + 1)]
    state = oracle.filter_frame(hosts[0], temporal=True, alpha_old=wl.alpha_old).state
    print(f"[bench] timing the oracle on {k} frames, one thread", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    nv = 0
    for i in range(1, k + 1):
        R = oracle.filter_frame(hosts[i], prev_state=state, temporal=True, alpha_old=wl.alpha_old)
        state = R.state
        nv += int(hosts[i]["valid"].sum())
    dt = time.perf_counter() - t0
    del hosts, state, R
    one = nv / dt
    w = workers or host_cores()
    per = 2
    print(f"[bench] timing the oracle in {w} host processes x {per} frames", file=sys.stderr, flush=True)
    ctx = mp.get_context("spawn")   # fresh interpreters: nothing of this process's GPU state is inherited
    barrier, results = ctx.Barrier(w), ctx.Queue()
    procs = [ctx.Process(target=_oracle_worker, args=(wl.name, (3 * j) % 13, per, barrier, results))
             for j in range(w)]
    for p in procs:
        p.start()
    got = [results.get(timeout=600) for _ in procs]
    for p in procs:
        p.join(timeout=60)
    span = max(t1 for _, t1, _ in got) - min(t0 for t0, _, _ in got)
    nv_all = sum(x for _, _, x in got)
    return {"value": round(nv_all / span, 1), "unit": "vertices/s", "cores": w, "kind": "oracle",
            "sample": f"{w} host processes, each the oracle on {per} consecutive frames of {wl.name} "
                      f"(1920x1080x3 slots each) with the moving average: {nv_all} valid vertices in {span:.1f} s",
            "cpu_model": cpu_model(), "host_cores_online": os.cpu_count(),
            "one_core": {"value": round(one, 1), "cores": 1,
                         "sample": f"{k} consecutive frames, {dt:.1f} s on one host thread"}}


if __name__ == "__main__":
    main()
