"""Tile-size autotuning of a rasterization step.

The screen-tile side (8, 16 or 32 pixels) trades per-tile traversal work
(a larger tile walks a longer triangle list for more pixels) against
per-tile overhead and load balance; the best choice depends on the triangle
size distribution and the resolution mix, so it is measured: every candidate
runs the caller's step a few times on the device and the fastest is kept.
Capacities need no tuning pass: every eager call sizes the tile lists and
the backward fragment regions from its own counts (with headroom), and the
static-capacity mode then reuses those sizes.

Results are cached per workload signature in the process, and in a JSON
file when SOUP_AUTOTUNE_CACHE names one.
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Callable, Dict, Iterable, Optional

TILES = (8, 16, 32)
_cache: Dict[str, dict] = {}


def signature(scene, views) -> str:
    """Workload key: triangle count, texture and MLP shape, view sizes."""
    h = hashlib.sha1()
    h.update(repr((int(scene.T), tuple(scene.feats.shape[1:]), tuple(scene.dims))).encode())
    h.update(views.widths.tobytes())
    h.update(views.heights.tobytes())
    return h.hexdigest()[:16]


def _file() -> Optional[str]:
    return os.environ.get("SOUP_AUTOTUNE_CACHE") or None


def _load_file() -> dict:
    f = _file()
    if not f or not os.path.exists(f):
        return {}
    try:
        with open(f) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(key: str, entry: dict) -> None:
    _cache[key] = entry
    f = _file()
    if not f:
        return
    data = _load_file()
    data[key] = entry
    tmp = f + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, f)


def cached(key: str) -> Optional[dict]:
    if key in _cache:
        return _cache[key]
    e = _load_file().get(key)
    if e is not None:
        _cache[key] = e
    return e


def cached_tile(key: str) -> Optional[int]:
    e = cached(key)
    return None if e is None else int(e["tile"])


def tune(step: Callable[[], None], ctx, key: str, tiles: Iterable[int] = TILES, reps: int = 3,
         force: bool = False) -> dict:
    """Time `step` (one full call sequence on ctx's stream) for every tile
    size and leave ctx set to the fastest. Returns {"tile", "ms": {tile: ms}}."""
    import torch
    if not force:
        e = cached(key)
        if e is not None:
            ctx.set_tile(int(e["tile"]))
            return e
    ms = {}
    for t in tiles:
        ctx.set_tile(int(t))
        step()   # sizes the workspaces for this tile
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            step()
        b.record()
        torch.cuda.synchronize()
        ms[int(t)] = a.elapsed_time(b) / reps
    best = min(ms, key=ms.get)
    ctx.set_tile(best)
    entry = {"tile": int(best), "ms": {str(k): round(v, 4) for k, v in ms.items()}}
    _store(key, entry)
    return entry
