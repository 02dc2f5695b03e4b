"""Autotuning of launch shapes and of the serving step, with a JSON cache of the winners.

Two knobs change how fast the renderer runs without changing any image:

* the launch shape of single-image renders: the shape of the pixel tile one wave marches (1x16 to
  16x1 pixels, 2^t wide) and the size of the super-tiles of such tiles dealt round-robin over the
  XCDs (2^(s+1) tiles on a side).  ``raypc_autotune_render`` times all 20 shapes on a view on the
  device and keeps the fastest; here its result is cached per device and workload class;
* the serving step: how many tiles one batched launch marches (``tiles_per_step``) and how many
  steps may be in flight at once (``steps_in_flight``).  ``tune_server`` replays a burst of
  requests through the public serving calls for each candidate and keeps the one that finishes
  the burst first.

The cache is a JSON object {key: winner}; keys name the device and the workload class (grid size,
storage, image size, level, step), so a winner is reused for renders of the same class.
"""
from __future__ import annotations

import json
import os
import time
from typing import Dict, Iterable, Optional, Sequence, Tuple

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "raypc", "autotune.json")

SERVER_CANDIDATES: Tuple[Tuple[int, int], ...] = ((8192, 2), (32768, 1), (32768, 2), (131072, 2))


def device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0) if torch.cuda.is_available() else "cpu"


def render_key(device: str, n: int, storage: str, width: int, height: int, lod: int, step: float) -> str:
    """Workload class of a single-image render."""
    return f"render|{device}|n{n}|{storage}|{width}x{height}|lod{lod}|step{step:g}"


def server_key(device: str, label: str) -> str:
    return f"server|{device}|{label}"


def load_cache(path: str = DEFAULT_CACHE) -> Dict[str, dict]:
    """The cached winners ({} when the file does not exist)."""
    try:
        with open(path) as f:
            data = json.load(f)
    except FileNotFoundError:
        return {}
    if not isinstance(data, dict):
        raise ValueError(f"{path}: not a JSON object")
    return data


def save_cache(cache: Dict[str, dict], path: str = DEFAULT_CACHE) -> None:
    """Write the cache atomically (a temporary file renamed over the old one)."""
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_render(rp, ctx, volume_id: int, camera, width: int, height: int, lod: int = 0, step: float = 0.5,
                repeats: int = 10, cache: Optional[Dict[str, dict]] = None, key: Optional[str] = None,
                retune: bool = False) -> dict:
    """Pick the launch shape for this view and make it the context's.  With a cache and a key, a
    cached winner is applied without timing (unless ``retune``); a new winner is stored in the cache
    (the caller saves it)."""
    if cache is not None and key is not None and key in cache and not retune:
        entry = cache[key]
        rp.set_launch_shape(ctx, int(entry["super_log2"]), int(entry["tile_log2w"]))
        return dict(entry, cached=True)
    (s, t), times = rp.autotune_render(ctx, volume_id, camera, width, height, lod, step, repeats)
    entry = {"super_log2": s, "tile_log2w": t, "wave_tile_px": [1 << t, 16 >> t],
             "super_tile_px": [(1 << t) << (s + 1), (16 >> t) << (s + 1)],
             "ms": times, "repeats": repeats}
    if cache is not None and key is not None:
        cache[key] = entry
    return dict(entry, cached=False)


def run_burst(rp, ctx, requests: Sequence, tiles_per_step: int, steps_in_flight: int, max_inflight: int = 64,
              mem_budget_bytes: int = 0) -> float:
    """Seconds from the first submission to the last completion of `requests` (all submitted at once)
    on a server started with the given step configuration."""
    import torch
    rp.server_start(ctx, mem_budget_bytes, max_inflight, tiles_per_step, steps_in_flight)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tickets = [rp.submit(ctx, r) for r in requests]
        for t in tickets:
            rp.wait(ctx, t, 60000)
        dt = time.perf_counter() - t0
        for t in tickets:
            rp.release(ctx, t)
    finally:
        rp.server_stop(ctx)
    return dt


def tune_server(rp, ctx, requests: Sequence, candidates: Iterable[Tuple[int, int]] = SERVER_CANDIDATES,
                rounds: int = 2, max_inflight: int = 64, mem_budget_bytes: int = 0,
                cache: Optional[Dict[str, dict]] = None, key: Optional[str] = None, retune: bool = False) -> dict:
    """Pick (tiles_per_step, steps_in_flight) for a request mix: each candidate serves the burst
    `rounds` times (after one untimed round) and the fastest median wins."""
    if cache is not None and key is not None and key in cache and not retune:
        return dict(cache[key], cached=True)
    results = []
    for tiles, steps in candidates:
        run_burst(rp, ctx, requests, tiles, steps, max_inflight, mem_budget_bytes)
        ts = sorted(run_burst(rp, ctx, requests, tiles, steps, max_inflight, mem_budget_bytes) for _ in range(rounds))
        results.append({"tiles_per_step": tiles, "steps_in_flight": steps, "s": ts[len(ts) // 2]})
    best = min(results, key=lambda r: r["s"])
    entry = {"tiles_per_step": best["tiles_per_step"], "steps_in_flight": best["steps_in_flight"],
             "requests": len(requests), "candidates": results}
    if cache is not None and key is not None:
        cache[key] = entry
    return dict(entry, cached=False)
