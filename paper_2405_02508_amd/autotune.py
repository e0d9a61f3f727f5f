"""Autotuner for the rasterizer's tile shape, small-triangle limit, large-
triangle limit and bin pool.

None of these change the results (the visibility rule is order-independent
and the overflow path is exact); they only change speed and workspace size.
For a view table and its geometry the tuner:
  1. runs mer_rasterize once per candidate and reads the number of
     triangle-tile entries from mer_status, so the bin pool can be sized to
     what the workload needs (plus a margin) instead of a worst case;
  2. times mer_rasterize for each candidate with HIP events on the current
     stream and keeps the fastest.
Choices are cached in a JSON file keyed by a shape class (view count,
pixel and triangle counts rounded to powers of two).
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

from . import mer

CANDIDATES = (
    # (tile_w, tile_h, small_px, big_tiles)
    (8, 8, 16, 16), (8, 8, 16, -1), (8, 8, 64, 16), (8, 8, 256, 16),
    (16, 16, 16, 16), (16, 16, 64, 16), (16, 16, 256, 16),
    (32, 8, 64, 16), (16, 8, 64, 16),
    (8, 8, -1, 16), (8, 8, -1, -1), (16, 16, -1, 16),
)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mer_autotune.json")


def shape_class(views_i64) -> str:
    V = np.asarray(views_i64, np.int64)
    px = int((V[:, 6] * V[:, 7]).sum())
    tris = int(V[:, 5].sum())
    b = lambda x: int(round(math.log2(max(x, 1))))  # noqa: E731
    return f"v2-v{V.shape[0]}-px2^{b(px)}-t2^{b(tris)}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(views_i64, v, tri, device="cuda", candidates=CANDIDATES, reps=3, cache_path=DEFAULT_CACHE,
         use_cache=True, log=None):
    """Return dict(tile=(w, h), small_px=int, big_tiles=int, bin_cap=int, ms=float, table=[...])."""
    import torch
    key = shape_class(views_i64)
    if use_cache and cache_path:
        hit = _load(cache_path).get(key)
        if hit:
            hit["tile"] = tuple(hit["tile"])
            hit["cached"] = True
            return hit
    n_px = int(mer.plan_init(views_i64).total_px)
    tid = torch.empty(n_px, dtype=torch.int32, device=device)
    depth = torch.empty(n_px, dtype=torch.float32, device=device)
    bary = torch.empty(n_px, 2, dtype=torch.float32, device=device)
    stream = torch.cuda.current_stream()
    table = []
    best = None
    for (tw, th, sp, bt) in candidates:
        ctx = mer.Context(views_i64, device=device, tile=(tw, th), small_px=sp, big_tiles=bt)
        ctx.rasterize(v, tri, tid, depth, bary)
        st = ctx.status()
        cap = int(st["entries"] * 1.25) + 4096
        del ctx
        ctx = mer.Context(views_i64, device=device, tile=(tw, th), small_px=sp, big_tiles=bt, bin_cap=cap)
        ctx.rasterize(v, tri, tid, depth, bary)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            ctx.rasterize(v, tri, tid, depth, bary)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        row = dict(tile=(tw, th), small_px=sp, big_tiles=bt, bin_cap=cap, entries=int(st["entries"]), ms=round(ms, 4))
        table.append(row)
        if log:
            log(f"[autotune] {row}")
        if best is None or ms < best["ms"]:
            best = row
        del ctx
        torch.cuda.empty_cache()
    out = dict(best, table=table, key=key, cached=False)
    if cache_path:
        data = _load(cache_path)
        data[key] = {k: out[k] for k in ("tile", "small_px", "big_tiles", "bin_cap", "entries", "ms")}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1)
        os.replace(tmp, cache_path)
    return out
