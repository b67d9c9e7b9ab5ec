"""Launch-parameter autotuner of the stroke-expansion pipeline.

The outline does not depend on the launch parameters (``sx_set_tuning``), only
the speed does: the slot kernel's register budget (waves per SIMD it must
allow; more waves hide more FP64 latency but spill more), the bisection
kernels' range of tags per wave and their register budget, and the number of
records per emission item chunk (work per record-kernel thread; longer chunks
amortise the item read, shorter ones balance the load).  The tuner times
candidates on the caller's own scene with HIP events on the caller's stream,
one knob group at a time (the groups drive different kernels), and keeps the
fastest; results are cached per device and workload shape in a JSON file so a
serving process tunes once.
"""
from __future__ import annotations

import json
import math
import os
import threading
from typing import Dict, Iterable, Optional, Tuple

PIECE_WAVES = (1, 2, 3)
BISECT_RANGE = (128, 192, 256, 384, 512, 1024)
BISECT_WAVES = (2, 3, 4)
CHUNK_K = (4, 8, 16, 32, 64)
KEYS = ("piece_waves", "chunk_k", "bisect_range", "bisect_waves")

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
                stream, reps: int = 5, counts=None) -> float:
    """Average ms of one asynchronous expansion with the context's current
    tuning, timed with HIP events on ``stream`` (after one untimed run).
    ``counts``: the device tensor behind count_ptr; when given, the untimed
    run's status is read and an item workspace too short for these launch
    parameters (smaller record chunks need more item units) is grown by one
    synchronous expansion before the timed runs, so that no candidate is
    timed on a run that stopped short."""
    import torch

    ctx.expand_async(scene, out_ptr, capacity, count_ptr, tolerance, mode, stream=stream)
    if counts is not None:
        stream.synchronize()
        if int(counts[1].item()) != 0:
            ctx.expand_into(scene, out_ptr, capacity, tolerance, mode, stream)
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
         reps: int = 5, cache_path: Optional[str] = None, use_cache: bool = True,
         counts=None) -> Tuple[dict, Dict[str, float]]:
    """Pick the fastest launch parameters for this scene and set them on
    ``ctx``.  The output buffer must already be large enough (size it with
    one ``ctx.expand``); pass the device tensor behind count_ptr as
    ``counts`` so that each candidate's item workspace is checked.  Coordinate search: the slot kernel's waves, then the
    bisection range and waves, then the chunk size.  Returns (chosen tuning,
    {"w{W}r{R}b{B}k{K}": ms} of every candidate timed; empty when the cache
    answered)."""
    import torch

    stream = stream if stream is not None else torch.cuda.current_stream()
    path = cache_path or default_cache_path()
    # the library runs on gfx950 only; the device's marketing name is not a
    # stable key (it differs between runtimes and profilers)
    key = workload_key("gfx950", scene.n_tags, mode, tolerance)
    if use_cache:
        with _lock:
            hit = _load(path).get(key)
        if (hit and all(k in hit for k in KEYS) and hit["piece_waves"] in PIECE_WAVES
                and hit["bisect_range"] in BISECT_RANGE and hit["bisect_waves"] in BISECT_WAVES
                and 1 <= int(hit["chunk_k"]) <= 255):
            ctx.set_tuning(**{k: int(hit[k]) for k in KEYS})
            return ctx.get_tuning(), {}
    times: Dict[str, float] = {}
    cur = ctx.get_tuning()

    def run(t):
        name = f"w{t['piece_waves']}r{t['bisect_range']}b{t['bisect_waves']}k{t['chunk_k']}"
        if name not in times:
            ctx.set_tuning(**t)
            times[name] = time_config(ctx, scene, tolerance, mode, out_ptr, capacity, count_ptr, stream, reps,
                                      counts=counts)
        return times[name]

    for group in ({"piece_waves": PIECE_WAVES}, {"bisect_range": BISECT_RANGE, "bisect_waves": BISECT_WAVES},
                  {"chunk_k": CHUNK_K}):
        names = list(group)
        cands = [dict(cur)]
        for vals in _product([group[n] for n in names]):
            c = dict(cur)
            c.update(zip(names, vals))
            cands.append(c)
        cur = min(cands, key=run)
    ctx.set_tuning(**cur)
    chosen = ctx.get_tuning()
    with _lock:
        data = _load(path)
        data[key] = dict(chosen, ms=min(times.values()))
        _store(path, data)
    return chosen, times


def _product(lists):
    if not lists:
        yield ()
        return
    for v in lists[0]:
        for rest in _product(lists[1:]):
            yield (v,) + rest
