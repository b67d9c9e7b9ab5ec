"""Launch-parameter autotuner of the stroke-expansion pipeline.

The outline does not depend on the launch parameters (``sx_set_tuning``), only
the speed does: the piece kernel's register budget (waves per SIMD it must
allow; more waves hide more FP64 latency but spill more), its workgroup size
(one wave per group frees a SIMD as soon as its wave ends) and the number of
records per emission item chunk (work per record-kernel thread; longer chunks
amortise the item read, shorter ones balance the load).  The tuner times each
candidate on the caller's own scene with HIP events on the caller's stream and
keeps the fastest; results are cached per device and workload shape in a JSON
file so a serving process tunes once.
"""
from __future__ import annotations

import json
import math
import os
import threading
from typing import Dict, Iterable, Optional, Tuple

PIECE_WAVES = (1, 2, 3)
PIECE_BLOCK = (64, 256)
CHUNK_K = (4, 8, 16, 32, 64)

_lock = threading.Lock()


def default_cache_path() -> str:
    base = os.environ.get("STROKEX_TUNE_CACHE")
    if base:
        return base
    return os.path.join(os.path.expanduser("~"), ".cache", "strokex", "tuning.json")


def workload_key(device_name: str, n_tags: int, mode: int, tolerance: float) -> str:
    """Cache key: device, output mode, tolerance and the scene size rounded to
    a power of two (the best parameters change slowly with size)."""
    size = 1 << max(0, int(math.log2(max(1, n_tags))))
    return f"{device_name}|mode{mode}|tol{tolerance:g}|tags~{size}"


def _load(path: str) -> Dict[str, dict]:
    try:
        with open(path, "r", encoding="utf-8") as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path: str, data: Dict[str, dict]) -> None:
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w", encoding="utf-8") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def time_config(ctx, scene, tolerance: float, mode: int, out_ptr: int, capacity: int, count_ptr: int,
                stream, reps: int = 5) -> float:
    """Average ms of one asynchronous expansion with the context's current
    tuning, timed with HIP events on ``stream`` (after one untimed run)."""
    import torch

    ctx.expand_async(scene, out_ptr, capacity, count_ptr, tolerance, mode, stream=stream)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    for _ in range(reps):
        ctx.expand_async(scene, out_ptr, capacity, count_ptr, tolerance, mode, stream=stream)
    t1.record(stream)
    t1.synchronize()
    return t0.elapsed_time(t1) / reps


def tune(ctx, scene, tolerance: float, mode: int, out_ptr: int, capacity: int, count_ptr: int, stream=None,
         waves: Iterable[int] = PIECE_WAVES, blocks: Iterable[int] = PIECE_BLOCK, chunks: Iterable[int] = CHUNK_K,
         reps: int = 5, cache_path: Optional[str] = None, use_cache: bool = True) -> Tuple[dict, Dict[str, float]]:
    """Pick the fastest (piece_waves, piece_block, chunk_k) for this scene and
    set it on ``ctx``.  The output buffer must already be large enough (size
    it with one ``ctx.expand``).  The piece-kernel knobs are searched first
    with the current chunk size, then the chunk size with the best of those
    (the two stages do not interact: chunk_k only changes the record kernel).
    Returns (chosen tuning, {"w{W}b{B}k{K}": ms} of every candidate timed;
    empty when the cache answered)."""
    import torch

    stream = stream if stream is not None else torch.cuda.current_stream()
    path = cache_path or default_cache_path()
    key = workload_key(torch.cuda.get_device_name(ctx.device), scene.n_tags, mode, tolerance)
    if use_cache:
        with _lock:
            hit = _load(path).get(key)
        if (hit and hit.get("piece_waves") in PIECE_WAVES and hit.get("piece_block") in PIECE_BLOCK
                and 1 <= int(hit.get("chunk_k", 0)) <= 255):
            ctx.set_tuning(int(hit["piece_waves"]), int(hit["chunk_k"]), int(hit["piece_block"]))
            return ctx.get_tuning(), {}
    times: Dict[str, float] = {}
    k0 = ctx.get_tuning()["chunk_k"]

    def run(w, b, k):
        ctx.set_tuning(w, k, b)
        ms = time_config(ctx, scene, tolerance, mode, out_ptr, capacity, count_ptr, stream, reps)
        times[f"w{w}b{b}k{k}"] = ms
        return ms

    best = min(((run(w, b, k0), w, b) for w in waves for b in blocks), key=lambda t: t[0])
    _, bw, bb = best
    bestk = min(((times.get(f"w{bw}b{bb}k{k}") or run(bw, bb, k), k) for k in chunks), key=lambda t: t[0])
    ctx.set_tuning(bw, bestk[1], bb)
    chosen = ctx.get_tuning()
    with _lock:
        data = _load(path)
        data[key] = dict(chosen, ms=bestk[0])
        _store(path, data)
    return chosen, times
