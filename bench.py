#!/usr/bin/env python
"""Benchmark of GPU stroke expansion on one MI355X.

Headline (``value``): input path segments expanded per second at 0.25 px
tolerance on the map/CAD-shaped scene (10,000 paths, 1,000,000 segments: 60%
lines, 15% quads, 25% cubics, mixed joins/caps, lognormal half-widths), line
output, plain per-scene expansion.  One step = the whole hot path over the
scene already resident in HBM: tag-monoid scan, bisection count pass, slot
scan, bisection write pass, piece and tail slot kernels (Euler spirals,
parallel curves, evolutes, joins and caps as emission items with record
counts), record-count scan, record kernel.

Beside it, in the same JSON line:
  * ``batched``: 256 map-shaped scenes (log-uniform 100..200k segments) in one
    graph-captured batched pipeline vs a loop of per-scene launches;
  * ``served``: Poisson arrivals into the continuous-batching server vs serial
    FIFO plain expansion, p50/p99 latency and throughput;
  * ``roofline`` of the dominant kernel and ``cpu_baseline`` (the FP64 oracle
    on the host cores, bounded sample).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6

# Algorithmic FP64 work per unit, counted from the definitions
# (transcendentals at the FMA count of their polynomial evaluation: sin/cos
# 25, sincos 40, atan2 40, acos 40, cbrt 30, sqrt 10, divide 10):
#   fit trial (Algorithm 2): sub-cubic end point, tangent and chord 70, two
#     end angles 92, arms 24, the Section 7.1 estimate 180, hodograph 91 = 460
#   line step: chord length and acceptance                               = 15
#   accepted cubic piece: the trial again 460, end normals 66, Appendix A
#     polynomials 50, Z(1) by 8-node quadrature (paired nodes) 226,
#     rotation and base angle 66, L 10                                  = 880
#   line piece: normal 33, length 13, angle 40                           = 90
#   parallel-curve range: curvatures, density split and its F increment
#     (Section 4.2 branches) or the arc count (Section 5), count           = 130
#   evolute bundle: Section 6 count and exact end points                  = 90
#   join or cap: tangents, normals, offsets, round-join angles            = 150
FLOPS = {"trial": 460.0, "line_step": 15.0, "piece": 880.0, "line": 90.0, "range": 130.0, "evolute": 90.0,
         "join": 150.0}
# Algorithmic FP32 work of the record kernel per output record (one new
# outline point per record): spiral position by 4-node quadrature 118,
# normal 24, offset 4, point placement (inverse of the density integral) 54
# for lines; arcs replace placement by the sweep and curvature 32.
FLOPS_PER_RECORD = {0: 200.0, 1: 178.0}
RECORD_BYTES = {0: 20, 1: 24}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sc, mode, budget_s=12.0):
    """The FP64 oracle (single thread, as it stands) on a bounded prefix of the
    same scene: whole tag ranges, grown until ~budget_s of CPU time."""
    import numpy as np

    import oracle as O

    enc = O.encode(sc)
    n_tags = len(enc.tags)
    t0 = time.process_time()
    w0 = time.time()
    done_tags = 0
    segs = 0
    recs = 0
    step = 20000
    while done_tags < n_tags and time.process_time() - t0 < budget_s:
        end = min(n_tags, done_tags + step)
        r = O.expand(sc, mode=mode, tag_begin=done_tags, tag_end=end, enc=enc)
        recs += len(r.out)
        segs += int(np.count_nonzero((enc.tags[done_tags:end] & 4) == 0))
        done_tags = end
    cpu = time.process_time() - t0
    wall = time.time() - w0
    return {
        "value": segs / wall,
        "unit": "input segs/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {done_tags} of {n_tags} tags ({segs} segments, {recs} records) of the same scene, "
                  f"{wall:.1f} s wall / {cpu:.1f} s CPU, FP64, single thread",
        "records_per_s": recs / wall,
        "cpu_model": _cpu_model(),
        "nproc": os.cpu_count(),
    }


# ------------------------------------------------------------------ plain
def roofline_of(phase_ms, stats, n_tags, n_rec, mode, names):
    """Roofline entry of the dominant phase and the achieved rate of every
    phase: algorithmic work per launch (per-unit figures times the unit
    counts of the instrumented run) over the average launch time."""
    n_slots = stats["pieces"] + n_tags
    curve_pieces = stats["pieces"] - stats["lines"]
    work = {
        # algorithmic FP64 flops per launch of each kernel
        "bisect_count": stats["trials"] * FLOPS["trial"] + stats["lines"] * FLOPS["line_step"],
        "pieces": (curve_pieces * FLOPS["piece"] + stats["lines"] * FLOPS["line"] + stats["ranges"] * FLOPS["range"]
                   + stats["evolutes"] * FLOPS["evolute"]),
        "tails": stats["joins"] * FLOPS["join"],
        # algorithmic FP32 flops
        "records": n_rec * FLOPS_PER_RECORD[mode],
        # algorithmic bytes
        "scan_tags": n_tags * 17.0,
        "scan_slots": n_tags * 12.0,
        "scan_records": n_slots * 12.0,
        # the write pass copies the kept piece codes into the canonical slot
        # array (a tag with more pieces than are kept re-runs its bisection)
        "bisect_write": n_slots * 8.0 + (n_slots - n_tags) * 4.0 + n_tags * 12.0,
    }
    dom = max(phase_ms, key=phase_ms.get)
    t_dom = phase_ms[dom] * 1e-3
    if dom in ("bisect_count", "pieces", "tails"):
        achieved = work[dom] / t_dom / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None, "precision": "fp64 (decisions)"}
    elif dom == "records":
        achieved = work[dom] / t_dom / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None}
    else:
        gbs = work[dom] / t_dom / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": gbs / PEAK_HBM_GBS, "traffic": None}
    roof["algorithmic_work_per_launch"] = work[dom]
    roof["phase_ms"] = phase_ms
    roof["work_counts"] = stats
    roof["flops_per_unit"] = FLOPS
    roof["flops_per_record"] = FLOPS_PER_RECORD[mode]
    roof["per_kernel"] = {
        n: ({"TFLOP/s": work[n] / (phase_ms[n] * 1e-3) / 1e12} if n in ("bisect_count", "pieces", "tails",
                                                                         "records")
            else {"GB/s": work[n] / (phase_ms[n] * 1e-3) / 1e9}) for n in names}
    return roof


def plain(args, ctx, B, S, torch, np):
    mode = S.OUT_LINES if args.mode == "lines" else S.OUT_ARCS
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    log("bench: generating the map scene")
    sc = S.scene_map(2, args.segments, args.paths, 0.25, mode)
    if args.fill_scene:
        sc = S.with_fills(sc)
    n_seg = sc.n_segments()
    scene = ctx.encode(sc, stream=stream)
    tol = sc.tolerance
    recs, n_rec, buf = ctx.expand(scene, tol, mode, stream=stream)  # sizes output and workspace
    cnt = torch.zeros(2, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    log(f"bench: {n_seg} segments, {scene.n_tags} tags -> {n_rec} records")

    tune_info = {}
    manual = {k: v for k, v in (("piece_waves", args.piece_waves), ("chunk_k", args.chunk_k),
                                ("bisect_range", args.bisect_range), ("bisect_waves", args.bisect_waves)) if v}
    if manual:
        ctx.set_tuning(**manual)
    elif not args.no_tune:
        from paper_2405_00127_amd import autotune as AT

        log("bench: autotuning launch parameters")
        _, times = AT.tune(ctx, scene, tol, mode, buf.data_ptr(), buf.numel(), cnt.data_ptr(), stream,
                           use_cache=False)
        tune_info = {"candidates_ms": times}
    tune_info["chosen"] = ctx.get_tuning()
    log(f"bench: tuning {tune_info['chosen']}")

    def step():
        ctx.expand_async(scene, buf.data_ptr(), buf.numel(), cnt.data_ptr(), tol, mode, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert int(cnt[0].item()) == n_rec and int(cnt[1].item()) == 0
    ms = (t1 - t0) * 1e3 / args.steps
    log(f"bench: plain {ms:.3f} ms/step")

    # per-kernel times: HIP events on the launching stream around each phase
    names = B.PHASE_NAMES
    nph = len(names)
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nph)]
           for _ in range(args.steps)]
    for k in range(args.steps):
        for p in range(nph):
            evs[k][p][0].record(stream)
            ctx.run_phase(scene, p, tol, mode, buf.data_ptr(), buf.numel(), stream=stream)
            evs[k][p][1].record(stream)
    torch.cuda.synchronize()
    phase_ms = {names[p]: sum(evs[k][p][0].elapsed_time(evs[k][p][1]) for k in range(args.steps)) / args.steps
                for p in range(nph)}
    log("bench: phases " + ", ".join(f"{n} {phase_ms[n]:.3f} ms" for n in names))
    stats = ctx.piece_stats(scene, tol, mode, stream=stream)
    log(f"bench: work {stats}")

    n_tags = scene.n_tags
    roof = roofline_of(phase_ms, stats, n_tags, n_rec, mode, names)
    out = {
        "metric": "path segs/s expanded at 0.25px tol (batched vs plain); p50/p99 request latency",
        "value": n_seg / (ms * 1e-3),
        "unit": "input segs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 decisions)",
        "data": "synthetic (seeded map/CAD-shaped scene; the paper's datasets are not available)",
        "config": {
            "workload": f"map/CAD scene, {args.paths} paths, {n_seg} segments (60% lines, 15% quads, 25% cubics), "
                        + ("every path filled, " if args.fill_scene else "")
                        + f"plain per-scene expansion, {args.mode}, tol 0.25 px",
            "segments": n_seg, "tags": n_tags, "records": n_rec, "output": args.mode, "tolerance": tol,
        },
        "output_records_per_s": n_rec / (ms * 1e-3),
        "roofline": roof,
        "tuning": tune_info,
    }
    return out, sc, mode


# ------------------------------------------------------------------- fill
def fill(args, ctx, B, S, torch, np):
    """The same map scene with every path filled (flattened at offset 0, one
    run per piece, subpaths closed, no joins or caps), launched with the
    tuning the plain leg chose."""
    mode = S.OUT_LINES if args.mode == "lines" else S.OUT_ARCS
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    sc = S.with_fills(S.scene_map(2, args.segments, args.paths, 0.25, mode))
    n_seg = sc.n_segments()
    scene = ctx.encode(sc, stream=stream)
    tol = sc.tolerance
    recs, n_rec, buf = ctx.expand(scene, tol, mode, stream=stream)
    cnt = torch.zeros(2, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()

    def step():
        ctx.expand_async(scene, buf.data_ptr(), buf.numel(), cnt.data_ptr(), tol, mode, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert int(cnt[0].item()) == n_rec and int(cnt[1].item()) == 0
    ms = (t1 - t0) * 1e3 / args.steps
    names = B.PHASE_NAMES
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in names]
           for _ in range(args.steps)]
    for k in range(args.steps):
        for p in range(len(names)):
            evs[k][p][0].record(stream)
            ctx.run_phase(scene, p, tol, mode, buf.data_ptr(), buf.numel(), stream=stream)
            evs[k][p][1].record(stream)
    torch.cuda.synchronize()
    phase_ms = {names[p]: sum(evs[k][p][0].elapsed_time(evs[k][p][1]) for k in range(args.steps)) / args.steps
                for p in range(len(names))}
    stats = ctx.piece_stats(scene, tol, mode, stream=stream)
    roof = roofline_of(phase_ms, stats, scene.n_tags, n_rec, mode, names)
    res = {
        "workload": f"map/CAD scene, {args.paths} paths, {n_seg} segments, every path filled, {args.mode}, "
                    f"tol 0.25 px",
        "segments": n_seg, "tags": scene.n_tags, "records": n_rec,
        "ms_per_step": ms, "segs_per_s": n_seg / (ms * 1e-3), "records_per_s": n_rec / (ms * 1e-3),
        "phase_ms": phase_ms,
        "roofline": {k: roof[k] for k in ("kernel", "bound", "achieved", "peak", "unit", "frac", "traffic",
                                          "algorithmic_work_per_launch", "per_kernel", "work_counts")},
    }
    log(f"bench: fill {ms:.3f} ms/step, {n_rec} records; phases "
        + ", ".join(f"{n} {phase_ms[n]:.3f}" for n in names))
    del buf
    return res, sc


# ---------------------------------------------------------------- batched
def batched(args, ctx, B, S, torch, np):
    """256 map-shaped scenes: one graph-captured batched pipeline vs a loop of
    one launch sequence per scene, same GPU, same stream, same outputs."""
    mode = S.OUT_LINES if args.mode == "lines" else S.OUT_ARCS
    tol = 0.25
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream()
    log("bench: generating the batch scenes")
    scs = S.scene_batch(4, args.batch_scenes, 100, 200_000, mode)
    sizes = [s.n_segments() for s in scs]
    total_seg = int(sum(sizes))
    scenes = [ctx.encode(s, stream=stream) for s in scs]
    # plain loop: each scene into its own slice of one buffer
    rec = B.RECORD_BYTES[mode]
    probe = torch.empty(16, dtype=torch.uint8, device=dev)
    counts = []
    for s in scenes:  # one synchronous call per scene sizes its item workspace and tells its record count
        try:
            counts.append(ctx.expand_into(s, probe.data_ptr(), 0, tol, mode, stream))
        except B.StrokexError as e:
            if e.code != B.SX_ETOOSMALL:
                raise
            counts.append(e.required)
    starts = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    total_rec = int(starts[-1])
    buf = torch.empty(max(1, total_rec) * rec, dtype=torch.uint8, device=dev)
    cnts = torch.zeros(2 * len(scenes), dtype=torch.int64, device=dev)

    def loop_step():
        for i, s in enumerate(scenes):
            ctx.expand_async(s, buf.data_ptr() + int(starts[i]) * rec, int(counts[i]) * rec,
                             cnts.data_ptr() + 16 * i, tol, mode, stream=stream)

    # batched: one arena, one pipeline, captured in a graph
    batch = B.Batch(ctx)
    batch.set(scenes, stream=stream)
    bout, boffs, bstatus = batch.prepare(tol, mode, stream=stream)

    def batch_step():
        batch.expand_async(tol, mode, bout.data_ptr(), bout.numel(), boffs.data_ptr(), bstatus.data_ptr(),
                           stream=stream)

    with torch.cuda.stream(stream):
        loop_step()
        batch_step()
    stream.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        batch_step()
    stream.synchronize()

    def timed(fn, k):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(stream)
        with torch.cuda.stream(stream):
            for _ in range(k):
                fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / k, e0.elapsed_time(e1) / k

    with torch.cuda.stream(stream):
        for _ in range(2):
            loop_step()
            g.replay()
    loop_ms, loop_dev = timed(loop_step, args.batch_steps)
    graph_ms, graph_dev = timed(lambda: g.replay(), args.batch_steps)
    # same outputs: every scene's records, bit for bit
    o = boffs.cpu().numpy()
    same = bool(np.array_equal(o, starts) and int(bstatus[1]) == 0
                and torch.equal(bout[: total_rec * rec], buf[: total_rec * rec]))
    del g
    batch.destroy()
    return {
        "workload": f"{len(scs)} map/CAD scenes, log-uniform 100..200k segments, {total_seg} segments, "
                    f"{args.mode}, tol 0.25 px",
        "segments": total_seg,
        "records": total_rec,
        "min_scene": int(min(sizes)),
        "max_scene": int(max(sizes)),
        "batched_graph_ms": graph_ms,
        "batched_segs_per_s": total_seg / (graph_ms * 1e-3),
        "plain_loop_ms": loop_ms,
        "plain_loop_segs_per_s": total_seg / (loop_ms * 1e-3),
        "speedup": loop_ms / graph_ms,
        "device_ms": {"batched": graph_dev, "plain_loop": loop_dev},
        "outputs_identical": same,
    }


# ----------------------------------------------------------------- served
def served(args, ctx, B, S, torch, np):
    from paper_2405_00127_amd import serve as V

    mode = S.OUT_LINES if args.mode == "lines" else S.OUT_ARCS
    tol = 0.25
    log("bench: generating the request pool")
    rng = np.random.Generator(np.random.PCG64(55))
    sizes = np.floor(np.exp(rng.uniform(math.log(1000), math.log(1_000_000), args.pool))).astype(int)
    scs = [S.scene_map(500 + i, int(n), max(1, int(n) // 100), tol, mode) for i, n in enumerate(sizes)]
    segs = [s.n_segments() for s in scs]
    pool = [ctx.encode(s) for s in scs]
    probe = torch.empty(16, dtype=torch.uint8, device="cuda:0")
    for s in pool:  # size each scene's item workspace (the serial baseline runs them alone)
        try:
            ctx.expand_into(s, probe.data_ptr(), 0, tol, mode)
        except B.StrokexError as e:
            if e.code != B.SX_ETOOSMALL:
                raise
    # one server for every load point; its slots are warmed first (arena and
    # workspace growth happen here, untimed)
    server = V.Server(ctx, tol, mode)
    V.run_load(ctx, pool, segs, 1e6, 4 * len(pool), tol, mode, seed=1, max_seconds=30.0, server=server)
    points = []
    for qps in args.qps:
        n = int(max(50, min(2000, qps * args.serve_seconds)))
        log(f"bench: serving at {qps} req/s ({n} requests)")
        srv = V.run_load(ctx, pool, segs, qps, n, tol, mode, seed=7, max_seconds=args.serve_seconds,
                         server=server)
        ser = V.run_serial(ctx, pool, segs, qps, n, tol, mode, seed=7, max_seconds=args.serve_seconds)
        points.append({"qps": qps, "served": srv, "serial_fifo": ser})
        log(f"bench:   served {srv}")
        log(f"bench:   serial {ser}")
    server.close()
    return {
        "workload": f"Poisson arrivals, requests log-uniform 1k..1M segments from a pool of {len(pool)} "
                    f"encoded map scenes (mean {np.mean(segs):.0f} segments), {args.mode}, tol 0.25 px",
        "points": points,
    }


def kernel_source_hash() -> str:
    """Hash of the HIP sources without comments and blank space: counter
    readings are tied to the code they were taken on."""
    import hashlib
    import re

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2405_00127_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, name), "r", encoding="utf-8") as f:
                text = f.read()
            text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
            text = re.sub(r"//[^\n]*", " ", text)
            text = " ".join(text.split())
            h.update(name.encode() + b"\0" + text.encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, mode: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's reading), or
    None when the summary is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_map1M_{mode}.json")
    try:
        with open(path, "r", encoding="utf-8") as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    if data.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = data.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def phase_of_kernel(name: str):
    """Pipeline phase of a rocprofv3 kernel name (None for other kernels and
    for the launch variants with work counters, which run only to count)."""
    import re

    simple = (("scan_tags_kernel", "scan_tags"), ("scan_counts_kernel", "scan_slots"),
              ("scan_counts_dev_kernel", "scan_records"), ("record_kernel", "records"), ("finish_kernel", "finish"))
    for key, phase in simple:
        if f"sx::{key}(" in name:
            return phase
    m = re.search(r"sx::bisect_kernel<(true|false), (true|false), \d+>", name)
    if m:
        return None if m.group(2) == "true" else ("bisect_write" if m.group(1) == "true" else "bisect_count")
    m = re.search(r"sx::slot_kernel<\d+, (true|false)>", name)
    if m:
        return None if m.group(1) == "true" else "pieces"
    m = re.search(r"sx::tail_kernel<(true|false)>", name)
    if m:
        return None if m.group(1) == "true" else "tails"
    return None


def summarize_counters(fetch_db: str, write_db: str, probe_mb: int, mode: str, commands) -> dict:
    """Per-launch HBM bytes of each phase from two rocprofv3 --pmc databases
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the same
    counter reads for the plain copy of probe_mb MiB that --copy-probe runs
    (the largest runtime copy kernel of the run)."""
    import sqlite3

    probe = float(probe_mb << 20)
    out = {"kernel_source_hash": kernel_source_hash(), "workload": f"map1M_{mode}", "commands": list(commands),
           "calibration": {"probe_bytes": probe}, "kernels": {}}
    per = {}
    for counter, db in (("FETCH_SIZE", fetch_db), ("WRITE_SIZE", write_db)):
        con = sqlite3.connect(db)
        rows = con.execute("select kernel_name, dispatch_id, value from counters_collection where counter_name = ?",
                           (counter,)).fetchall()
        con.close()
        copies = [v for k, _, v in rows if "copyBuffer" in k]
        if not copies:
            raise SystemExit(f"{db}: no copy kernel to calibrate {counter} against (run with --copy-probe)")
        factor = probe / (max(copies) * 1024.0)
        out["calibration"][counter] = {"copy_kib": max(copies), "factor": factor}
        for k, d, v in rows:
            ph = phase_of_kernel(k)
            if ph is not None:
                per.setdefault(ph, {}).setdefault(counter, {})[d] = v * 1024.0 * factor
    for ph, c in per.items():
        if "FETCH_SIZE" in c and "WRITE_SIZE" in c:
            f = sum(c["FETCH_SIZE"].values()) / len(c["FETCH_SIZE"])
            w = sum(c["WRITE_SIZE"].values()) / len(c["WRITE_SIZE"])
            out["kernels"][ph] = {"fetch_bytes": f, "write_bytes": w, "bytes_per_launch": f + w,
                                  "dispatches": [len(c["FETCH_SIZE"]), len(c["WRITE_SIZE"])]}
    return out


def summarize_valu(db: str, n_cu: int = 256, n_xcd: int = 8):
    """Per phase, from one rocprofv3 --pmc database with SQ_INSTS_VALU,
    SQ_ACTIVE_INST_VALU, SQ_THREAD_CYCLES_VALU, SQ_INSTS_SALU,
    SQ_INSTS_VALU_TRANS_F64 and GRBM_GUI_ACTIVE: VALU busy (share of the CUs'
    cycles issuing VALU work: ACTIVE_INST_VALU / (CUs x GUI cycles), GUI
    cycles = GRBM_GUI_ACTIVE summed over the XCDs / XCDs) and VALU lane
    utilisation (THREAD_CYCLES_VALU / (64 x ACTIVE_INST_VALU)), averaged over
    dispatches."""
    import sqlite3

    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, dispatch_id, counter_name, value from counters_collection").fetchall()
    con.close()
    per = {}
    for k, d, c, v in rows:
        ph = phase_of_kernel(k)
        if ph is not None:
            per.setdefault(ph, {}).setdefault(d, {})[c] = per.get(ph, {}).get(d, {}).get(c, 0.0) + v
    out = {}
    for ph, ds in per.items():
        def avg(c):
            return sum(x.get(c, 0.0) for x in ds.values()) / len(ds)

        gui = avg("GRBM_GUI_ACTIVE") / n_xcd
        act = avg("SQ_ACTIVE_INST_VALU")
        out[ph] = {"dispatches": len(ds), "gui_cycles": gui,
                   "valu_busy_pct": 100.0 * act / (n_cu * gui) if gui else None,
                   "valu_lane_util_pct": 100.0 * avg("SQ_THREAD_CYCLES_VALU") / (64.0 * act) if act else None,
                   "valu_insts": avg("SQ_INSTS_VALU"), "salu_insts": avg("SQ_INSTS_SALU"),
                   "valu_trans_f64_insts": avg("SQ_INSTS_VALU_TRANS_F64")}
    return out


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-valu":
        # offline: bench.py --summarize-valu DB
        print(json.dumps(summarize_valu(sys.argv[2]), indent=1))
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-counters":
        # offline: bench.py --summarize-counters FETCH_DB WRITE_DB PROBE_MB MODE [COMMAND ...]
        fetch_db, write_db, probe_mb, mode = sys.argv[2:6]
        res = summarize_counters(fetch_db, write_db, int(probe_mb), mode, sys.argv[6:])
        path = os.path.join(ROOT, "profiles", f"traffic_map1M_{mode}.json")
        with open(path, "w", encoding="utf-8") as f:
            json.dump(res, f, indent=1)
        print(json.dumps(res["kernels"], indent=1))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["lines", "arcs"], default="lines")
    ap.add_argument("--segments", type=int, default=1_000_000)
    ap.add_argument("--paths", type=int, default=10_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-parameter autotuner")
    ap.add_argument("--piece-waves", type=int, default=None)
    ap.add_argument("--chunk-k", type=int, default=None)
    ap.add_argument("--bisect-range", type=int, default=None)
    ap.add_argument("--bisect-waves", type=int, default=None)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-fill", action="store_true", help="skip the fill leg (the map scene filled)")
    ap.add_argument("--fill-scene", action="store_true",
                    help="time the map scene with every path filled in the main leg (for profiling the fill)")
    ap.add_argument("--batch-scenes", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--pool", type=int, default=64)
    ap.add_argument("--qps", type=float, nargs="*", default=[100.0, 1000.0, 5000.0])
    ap.add_argument("--serve-seconds", type=float, default=4.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="also run one plain device copy of this many MB (a known-size reference for "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only (asked for --gpus {args.gpus}); stroke expansion shards by "
              "scene, or for one scene by path ranges", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2405_00127_amd import binding as B
    from paper_2405_00127_amd import build as PB
    from paper_2405_00127_amd import scenes as S

    if not os.path.exists(B.LIB_PATH):
        PB.build()
    torch.cuda.set_device(0)
    ctx = B.Context(0)
    if args.copy_probe:
        n = args.copy_probe << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out, sc, mode = plain(args, ctx, B, S, torch, np)
    # the stored counters are those of the stroked map scene
    traffic = None if args.fill_scene else measured_traffic(out["roofline"]["kernel"], args.mode)
    if traffic is not None:
        out["roofline"]["traffic"] = traffic
    fill_sc = None
    if not args.no_fill:
        out["fill"], fill_sc = fill(args, ctx, B, S, torch, np)
    if not args.no_batched:
        out["batched"] = batched(args, ctx, B, S, torch, np)
        log(f"bench: batched {out['batched']}")
    if not args.no_served:
        out["served"] = served(args, ctx, B, S, torch, np)
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(sc, mode, args.cpu_budget)
        if fill_sc is not None:
            out["fill"]["cpu_baseline"] = cpu_baseline(fill_sc, mode, min(args.cpu_budget, 6.0))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
