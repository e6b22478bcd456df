"""Autotuner of batched Top-K plans.

A batched plan has free choices that trade launch work against streaming
efficiency and survivor traffic:

* ``tile_keys``      keys each filter workgroup streams (the block tile: how
                     many workgroups a query's pass is cut into);
* ``sample_sigma`` / ``max_sample_log2``
                     how far above the expected survivor count the sampled
                     threshold sits, and the largest sample: these size the
                     survivor buffers and decide how often the exact fallback
                     (a second pass over a query) runs;
* ``cap_sigma``      the survivor buffers' margin over the expected count;
* ``filter_grid``    filter workgroups looping over all the slices (0: three
                     per CU; 0xFFFFFFFF: one workgroup per slice).

``tune()`` times every candidate on the caller's own batch (each run is a
full, exact ``tk_plan_launch``; the tuner never changes a result, only how
fast it arrives) and returns the fastest.  ``cached_params()`` keeps winners
in a JSON file keyed by device name and key type, so a serving process tunes
once.  Candidate generation and the cache are plain Python and run anywhere;
timing needs the GPU.
"""

from __future__ import annotations

import itertools
import json
import os
import time

import numpy as np

DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned_plans.json")
ONE_PER_SLICE = 0xFFFFFFFF  # filter_grid: one filter workgroup per slice


def candidates(key_bytes: int, quick: bool = False):
    """Parameter sets to try, as dicts of tk_plan_params fields."""
    tiles = ([1 << 14, 1 << 15, 1 << 16, 1 << 17] if key_bytes == 8 else
             [1 << 15, 1 << 16, 1 << 17, 1 << 18])
    sigmas = [(4.0, 14), (3.0, 14), (4.0, 16), (4.0, 20)]
    caps = [6.0, 4.0]
    grids = [0, ONE_PER_SLICE]
    if quick:
        tiles, sigmas, caps, grids = tiles[1:3], sigmas[:2], caps[:1], grids
    return [{"tile_keys": t, "sample_sigma": s, "max_sample_log2": m, "cap_sigma": c,
             "filter_grid": g}
            for t, (s, m), c, g in itertools.product(tiles, sigmas, caps, grids)]


def _key(device_name: str, key_dtype: str) -> str:
    return f"{device_name}|{key_dtype}"


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def store(device_name: str, key_dtype: str, params: dict, seconds: float,
          path: str = DEFAULT_CACHE) -> None:
    d = load_cache(path)
    d[_key(device_name, key_dtype)] = {"params": params, "seconds": seconds,
                                       "tuned_at": time.strftime("%Y-%m-%dT%H:%M:%S")}
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def cached_params(device_name: str, key_dtype: str, path: str = DEFAULT_CACHE):
    e = load_cache(path).get(_key(device_name, key_dtype))
    return None if e is None else dict(e["params"])


def tune(offsets, ks, orders, keys, rid_dtype=None, reps: int = 3, quick: bool = False,
         stream=None, cache_path: str | None = DEFAULT_CACHE, log=None):
    """Times each candidate plan on this batch; returns (best params, seconds, table)."""
    import torch

    from .batched import Plan

    rid_dtype = rid_dtype or torch.uint32
    s = stream or torch.cuda.Stream()
    table = []
    best = None
    for p in candidates(keys.element_size(), quick):
        plan = Plan(offsets, ks, orders, key_dtype=keys.dtype, rid_dtype=rid_dtype, stream=s, **p)
        ok, orr = plan.alloc_outputs()
        torch.cuda.synchronize()
        plan.launch(keys, ok, orr, stream=s)  # eager first launch
        plan.launch(keys, ok, orr, stream=s)  # graph capture, outside the timing
        torch.cuda.synchronize()
        times = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            plan.launch(keys, ok, orr, stream=s)
            e1.record(s)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
        st = plan.stats()
        plan.close()
        t = float(np.median(times))
        table.append({**p, "seconds": t, "fallbacks": st["fallbacks"]})
        if log:
            log(table[-1])
        if best is None or t < best[1]:
            best = (p, t)
    if cache_path:
        store(torch.cuda.get_device_name(), str(keys.dtype).replace("torch.", ""), best[0], best[1],
              cache_path)
    return best[0], best[1], table
