"""Benchmark: hashed path space filtering of the 1080p x3 workload on one GPU.

One step filters one frame of the orbiting camera (1920x1080 pixels, 3 path
vertices per pixel, 6,220,800 vertex slots): clear the current table, build
keys, insert-accumulate, temporal moving average against the previous
frame's table, look up.  Sixteen frames are generated on the GPU before
timing (inputs resident in HBM) and steps cycle through them.

Prints one JSON line.  `value` is vertices filtered per second (valid
vertices, i.e. those with a hit, over the whole timed region); per-kernel
times come from HIP events on the stream the kernels run on.
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
    p.add_argument("--frames", type=int, default=16)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-frames", type=int, default=8, help="frames of the oracle timed on the host")
    return p.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on exactly one GPU (the filter has no multi-GPU path); got --gpus {a.gpus}",
              file=sys.stderr)
        sys.exit(2)
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

    flt = pf.FrameFilter(n, view.log2_slots, wl.max_probe, wl.frac_bits, temporal=True, alpha_old=wl.alpha_old,
                         agg_width=a.agg, device=dev)
    outs = (torch.empty(n, device=dev), torch.empty(n, device=dev), torch.empty(n, device=dev))
    stream = torch.cuda.current_stream()

    names = ["clear", "build_keys", "insert_accumulate", "temporal_update", "query_average"]

    def step(k, ev=None):
        f = frames[k % len(frames)]
        key, vflags, slot = flt.key[:n], flt.vflags[:n], flt.slot[:n]
        cur = flt.cur
        if ev is not None:
            ev[0].record(stream)
        pf.clear(cur)
        if ev is not None:
            ev[1].record(stream)
        pf.build_keys(f["px"], f["py"], f["pz"], f["nx"], f["ny"], f["nz"], f["valid"], f["cam"], f["s"],
                      f["seed"], 0, view.log2_slots, key, None, None, vflags)
        if ev is not None:
            ev[2].record(stream)
        pf.insert_accumulate(cur, key, f["r"], f["g"], f["b"], vflags, slot, a.agg)
        if ev is not None:
            ev[3].record(stream)
        pf.temporal_update(cur, flt.prev, wl.alpha_old)
        if ev is not None:
            ev[4].record(stream)
        pf.query_average(cur, key, slot, f["r"], f["g"], f["b"], vflags, True, outs[0], outs[1], outs[2], None)
        if ev is not None:
            ev[5].record(stream)
        flt.tables.reverse()
        flt.frames += 1

    print(f"[bench] warmup {a.warmup} steps", file=sys.stderr, flush=True)
    for k in range(a.warmup):
        step(k)
    torch.cuda.synchronize()

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(a.steps)]
    print(f"[bench] timing {a.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        step(a.warmup + k, events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = events[0][0].elapsed_time(events[-1][5])
    per = {nm: float(np.mean([events[k][j].elapsed_time(events[k][j + 1]) for k in range(a.steps)])) * 1e3
           for j, nm in enumerate(names)}  # microseconds
    valid_total = sum(n_valid[(a.warmup + k) % len(frames)] for k in range(a.steps))
    ms_per_step = wall * 1e3 / a.steps
    value = valid_total / wall

    # statistics of the last frame (untimed): cells, displacement, temporal hits
    st = pf.read_stats(flt.prev)
    cells = int(st[pf.STAT_USED])

    # quality: RMSE against the noise-free radiance over valid vertices (evaluation only)
    def rmse(x, f):
        v = f["valid"].bool()
        est = torch.stack(x, 1)[v]
        return float(torch.sqrt(((est - f["truth"][v]) ** 2).mean()))
    f_last = frames[(a.warmup + a.steps - 1) % len(frames)]
    q_temporal = rmse(outs, f_last)
    q_noisy = rmse((f_last["r"], f_last["g"], f_last["b"]), f_last)
    plain = pf.FrameFilter(n, view.log2_slots, wl.max_probe, wl.frac_bits, temporal=False, agg_width=a.agg,
                           device=dev)
    o2 = plain.filter(f_last["px"], f_last["py"], f_last["pz"], f_last["nx"], f_last["ny"], f_last["nz"],
                      f_last["valid"], f_last["r"], f_last["g"], f_last["b"], f_last["cam"], f_last["s"],
                      f_last["seed"])
    q_plain = rmse(o2, f_last)

    # roofline of the dominant kernel: algorithmic bytes per launch / mean launch time
    nv = float(np.mean(n_valid))
    algo_bytes = {
        "clear": cells * 32 + (1 << view.log2_slots) // 8,
        "build_keys": n * (6 * 4 + 1 + 8 + 1),
        "insert_accumulate": n * (1 + 4) + nv * (8 + 12 + 4 + 28),
        "temporal_update": cells * (32 + 8 + 4 + 8 + 16 + 16) + (1 << view.log2_slots) // 8,
        "query_average": n * (1 + 12) + nv * (4 + 16) + (n - nv) * 12,
    }
    dom = max(per, key=lambda k: per[k])
    achieved = algo_bytes[dom] / (per[dom] * 1e-6) / 1e9
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "algorithmic_bytes_per_launch": int(algo_bytes[dom])}

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(frames, wl, a.cpu_frames)

    line = {
        "metric": "vertices/s filtered (insert+query) at 1080p; RMSE vs noise-free mean",
        "value": round(value, 1), "unit": "vertices/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "fp32+int64", "data": "synthetic",
        "config": {"workload": a.workload, "width": view.width, "height": view.height,
                   "verts_per_path": view.verts_per_path, "vertex_slots": n, "valid_vertices_mean": round(nv, 1),
                   "log2_slots": view.log2_slots, "max_probe": wl.max_probe, "frac_bits": wl.frac_bits,
                   "frames": a.frames, "alpha_old": wl.alpha_old, "agg_width": a.agg, "parallelism": "single-gpu"},
        "vertex_slots_per_s": round(n * a.steps / wall, 1),
        "gpu_ms_per_step": round(gpu_ms / a.steps, 4),
        "insert_query_vertices_per_s": round(nv / ((per["insert_accumulate"] + per["query_average"]) * 1e-6), 1),
        "kernel_us": {k: round(v, 2) for k, v in per.items()},
        "cells_last_frame": cells,
        "rmse": {"unfiltered": round(q_noisy, 5), "filtered": round(q_plain, 5), "filtered_temporal": round(q_temporal, 5)},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def cpu_baseline(frames, wl, k):
    """The oracle (single-threaded C plus numpy glue) on k frames of the same
    workload, with the moving average; vertices/s over valid vertices."""
    import oracle
    hosts = [{kk: (v.cpu() if hasattr(v, "cpu") else v) for kk, v in frames[i].items()} for i in range(k + 1)]
    state = oracle.filter_frame(hosts[0], temporal=True, alpha_old=wl.alpha_old).state
    print(f"[bench] timing the oracle on {k} frames", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    nv = 0
    for i in range(1, k + 1):
        R = oracle.filter_frame(hosts[i], prev_state=state, temporal=True, alpha_old=wl.alpha_old)
        state = R.state
        nv += int(hosts[i]["valid"].sum())
    dt = time.perf_counter() - t0
    return {"value": round(nv / dt, 1), "unit": "vertices/s", "cores": 1, "kind": "oracle",
            "sample": f"{k} consecutive frames of {wl.name} (1920x1080x3 slots each) with the moving average, "
                      f"{dt:.1f} s on one host thread"}


if __name__ == "__main__":
    main()
