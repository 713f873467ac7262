"""Launch-shape autotuner for the persistent page decoder.

Times every candidate (sub-tile width x height in passes, waves per CU) on a page workload
with HIP events and keeps the fastest.  Results are cached in a JSON file keyed by device
name, CU count and workload class, and applied through ndgi_set_launch.
"""
from __future__ import annotations

import json
import os

from . import ndgi as N

CANDIDATES = [(tw, th, wpc) for tw in (1, 2) for th in (2, 4, 8, 16) for wpc in (12, 16, 32)]
CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")


def _key(torch, workload: str) -> str:
    p = torch.cuda.get_device_properties(0)
    return f"{p.name}|{p.multi_processor_count}|{workload}"


def tune_pages(ctx: N.Context, run, workload: str, reps: int = 5, candidates=CANDIDATES, use_cache=True):
    """Pick the fastest launch shape for `run()` (one page-decode launch on the current
    stream) and apply it to `ctx`.  Returns (shape, {shape: ms})."""
    import torch
    key = _key(torch, workload)
    cache = {}
    if use_cache and os.path.exists(CACHE):
        try:
            cache = json.load(open(CACHE))
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        shape = tuple(cache[key]["shape"])
        ctx.set_launch(*shape)
        return shape, cache[key].get("timings", {})
    timings = {}
    for shape in candidates:
        try:
            ctx.set_launch(*shape)
        except N.NdgiError:
            continue
        run()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            run()
            b.record()
        torch.cuda.synchronize()
        ms = sorted(a.elapsed_time(b) for a, b in ev)[reps // 2]
        timings[",".join(map(str, shape))] = ms
    best = min(timings, key=timings.get)
    shape = tuple(int(v) for v in best.split(","))
    ctx.set_launch(*shape)
    cache[key] = {"shape": list(shape), "timings": timings}
    try:
        with open(CACHE, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    except OSError:
        pass
    return shape, timings
