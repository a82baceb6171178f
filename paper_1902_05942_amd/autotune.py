"""Autotuner of the multi-view calls.

Times pf_filter_views for every (workgroup size, aggregation width) pair on
the caller's actual views and frames, keeps the fastest, and caches the
choice in a JSON file keyed by the device (name, compute units) and the
views' shapes; tune_streams times pf_filter_views_concurrent for 1 .. 3
library streams.  Every configuration computes identical results; only the
time differs.
"""
from __future__ import annotations

import json
import os

import torch

BLOCKS = (64, 128, 256, 512, 1024)
# aggregation width as a multiple of the workgroup size: 0 = device atomics
# per vertex; f > 0 = windows of f x block consecutive vertices merged by key
# in LDS before their cells are touched
AGG_FACTORS = (0, 1, 2, 4, 8)


def candidates(blocks=BLOCKS, factors=AGG_FACTORS):
    """Every (block, agg_width) pair the tuner times."""
    return [(b, f * b) for b in blocks for f in factors]


def cache_path() -> str:
    return os.environ.get("PF_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "pf_autotune.json"))


def signature(frames) -> str:
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    shapes = ",".join(str(f["px"].numel()) for f in frames)
    return f"{props.name}|{props.multi_processor_count}|{shapes}"


def time_config(mvf, frames, block, agg, reps=5) -> float:
    """Median milliseconds of one launch over `reps` launches after a warm-up."""
    mvf.filter(frames, block, agg)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        mvf.filter(frames, block, agg)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def tune(mvf, frames, blocks=BLOCKS, factors=AGG_FACTORS, reps=5, use_cache=True, verbose=False):
    """Returns (block, agg_width, {(block, agg): ms})."""
    key = signature(frames)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as fh:
                cache = json.load(fh)
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            c = cache[key]
            return c["block"], c["agg"], {tuple(map(int, k.split("/"))): v for k, v in c["ms"].items()}
    res = {}
    for b, a in candidates(blocks, factors):
        res[(b, a)] = time_config(mvf, frames, b, a, reps)
        if verbose:
            print(f"[autotune] block {b:4d} agg {a:4d}: {res[(b, a)]:.3f} ms", flush=True)
    best = min(res, key=res.get)
    if use_cache:
        cache[key] = {"block": best[0], "agg": best[1], "ms": {f"{b}/{a}": v for (b, a), v in res.items()}}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(cache, fh, indent=1)
        os.replace(tmp, path)
    return best[0], best[1], res


STREAMS = (1, 2, 3)


def tune_streams(mvf, frames, choices=STREAMS, reps=5):
    """For a MultiViewFilter in mode "concurrent": (fastest stream count,
    {streams: median ms})."""
    res = {}
    for ns in choices:
        mvf.filter(frames, nstreams=ns)
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            mvf.filter(frames, nstreams=ns)
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ts.sort()
        res[ns] = ts[len(ts) // 2]
    return min(res, key=res.get), res
