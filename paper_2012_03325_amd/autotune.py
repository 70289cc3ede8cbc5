"""Launch-schedule autotuner of batched frames.

A batch's schedule (shading tile, SSAO tile, SSAO gathers in flight,
workgroups per CU, seven stage launches or one persistent launch and its work
item size, bloom level 1 in the shading stage or not) changes only the speed of
epb_render_batch, never its results, so it can be picked by measurement alone.  The tuner runs a
coordinate descent over the schedule space: starting from the current best,
it tries every value of one parameter with the others held, keeps the fastest
(median of HIP-event timings over a few renders) and moves to the next
parameter, for a given number of passes.

Results are cached per batch signature (device, storage types, blur flag and
the multiset of view sizes and SSAO kernel lengths) in a process-wide table
guarded by a lock, optionally mirrored in a JSON file.
"""
from __future__ import annotations

import collections
import json
import os
import threading
from typing import Callable, Dict, List, Optional, Tuple

import torch

from . import epb as E

SPACE: Dict[str, Tuple[int, ...]] = {
    "blocks_per_cu": (0, 1, 2, 4, 8),
    "shade_tile": (0, 1, 2),
    "ssao_tile": (0, 1, 2),
    "ssao_batch": (0, 1),
    "persistent": (0, 16, 64, 256, 1024),
    "fuse_bloom": (0, 1),
}
ORDER = ("blocks_per_cu", "shade_tile", "ssao_tile", "ssao_batch", "persistent", "fuse_bloom")

_lock = threading.Lock()
_cache: Dict[str, Dict[str, int]] = {}


def _as_dict(s: E.epb_schedule) -> Dict[str, int]:
    return {k: int(getattr(s, k)) for k in ORDER}


def _as_sched(d: Dict[str, int]) -> E.epb_schedule:
    return E.epb_schedule(d["shade_tile"], d["ssao_tile"], d["ssao_batch"], d["blocks_per_cu"],
                          d.get("persistent", 0), 0, d.get("fuse_bloom", 0))


def signature(batch, device: Optional[str] = None) -> str:
    dv0 = batch.dviews[0]
    sizes = collections.Counter((dv.W, dv.H, int(dv.ssao_params.n_samples), len(dv.lights))
                                for dv in batch.dviews)
    key = dict(device=device if device is not None else torch.cuda.get_device_name(), g=dv0.gdtype,
               a=dv0.ao_dtype, h=dv0.hdr_dtype,
               blur=int(dv0.ssao_params.blur),
               views=sorted([list(k) + [c] for k, c in sizes.items()]))
    return json.dumps(key, sort_keys=True)


def time_render(batch, reps: int = 3, stream=None) -> float:
    """Median milliseconds of one batched render (after one untimed render)."""
    s = stream or torch.cuda.current_stream()
    batch.render(s)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record(s)
    for k in range(reps):
        batch.render(s)
        ev[k + 1].record(s)
    torch.cuda.synchronize()
    ms = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(reps))
    return ms[len(ms) // 2]


def tune(batch, reps: int = 3, passes: int = 2, cache_path: Optional[str] = None,
         use_cache: bool = True, timer: Optional[Callable] = None,
         device: Optional[str] = None) -> Tuple[E.epb_schedule, List[dict]]:
    """Pick the fastest schedule for ``batch`` (a frame.DeviceBatch) and leave
    the batch built with it.  Returns the schedule and the timings tried.
    ``timer(batch, reps)`` measures one schedule (default: HIP events around
    renders); ``device`` names the device in the cache key (default: the
    current GPU's name)."""
    timer = timer or time_render
    sig = signature(batch, device)
    if use_cache:
        with _lock:
            if not _cache and cache_path and os.path.exists(cache_path):
                with open(cache_path) as f:
                    _cache.update(json.load(f))
            hit = _cache.get(sig)
        if hit is not None:
            best = _as_sched(hit)
            batch.build(best)
            return best, [dict(schedule=hit, ms=None, cached=True)]
    tried: Dict[Tuple[int, ...], float] = {}
    trace: List[dict] = []

    def cost(d: Dict[str, int]) -> float:
        key = tuple(d[k] for k in ORDER)
        if key not in tried:
            try:
                batch.build(_as_sched(d))
            except E.EpbError as e:  # a schedule this batch cannot take (e.g. persistent with mixed storage)
                tried[key] = float("inf")
                trace.append(dict(schedule=dict(d), ms=None, rejected=str(e)))
                return tried[key]
            ms = timer(batch, reps)
            if d.get("persistent") and batch.status() != E.EPB_OK:  # a wait gave up: not a valid render
                tried[key] = float("inf")
                trace.append(dict(schedule=dict(d), ms=None, rejected="a persistent wait gave up"))
                return tried[key]
            tried[key] = ms
            trace.append(dict(schedule=dict(d), ms=ms))
        return tried[key]

    best = _as_dict(batch.schedule)
    best_ms = cost(best)
    for _ in range(passes):
        moved = False
        for k in ORDER:
            for v in SPACE[k]:
                cand = dict(best, **{k: v})
                ms = cost(cand)
                if ms < best_ms:
                    best, best_ms, moved = cand, ms, True
        if not moved:
            break
    batch.build(_as_sched(best))
    with _lock:
        _cache[sig] = best
        if cache_path:
            tmp = cache_path + ".tmp"
            with open(tmp, "w") as f:
                json.dump(_cache, f, indent=1, sort_keys=True)
            os.replace(tmp, cache_path)
    return _as_sched(best), trace
