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
# vector ALU, unpacked (the library is built without packed FP32): 256 CUs x
# 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz, the same for FP32 and FP64
PEAK_VALU_TFLOPS = 78.6
# VALU issue: a wave64 VALU instruction occupies a 16-lane SIMD for 4 clocks
# (the same 16 lanes x 2 flops per clock that give the flop peak), so at most
# 256 CUs x 4 SIMDs x 2.4 GHz / 4 wave instructions per second
PEAK_VALU_WAVE_INSTS = 256 * 4 * 2.4e9 / 4

# Algorithmic work per unit, in flop equivalents: an FMA counts 2, a
# transcendental (sin, cos, atan2, sqrt, cbrt, asin, pow, a division) 1.
#   fit trial (Algorithm 2, Section 7.1): 60 FMA + 7 transcendentals        = 127
#   output point (record kernel, one new outline point per record): inverse
#     of the density integral, map to u, Euler spiral position by a 4-node
#     quadrature, tangent, offset: 100 FMA + 10 transcendentals             = 210
#   accepted curve piece (piece kernel): its trial's chord and end angles
#     127, Appendix A polynomials 20 FMA (40), Z(1) by 4 nodes (4 sincos +
#     16 FMA: 40), end normals 10, L = chord / c 1                          = 218
#   line piece: chord length and normal, 8 FMA + 2 transcendentals           = 18
#   parallel-curve range (count of Section 4.2 or 5): 12 FMA + 4 trans.      = 28
#   evolute bundle (count of Section 6): 4 FMA + 4 transcendentals           = 12
#   join or cap (Algorithm 1): unit tangents, cross and dot, offsets, round
#     count: 10 FMA + 7 transcendentals                                     = 27
WORK = {"trial": 127.0, "point": 210.0, "piece": 218.0, "line": 18.0, "range": 28.0, "evolute": 12.0,
        "join": 27.0}
RECORD_BYTES = {0: 20, 1: 24}
ALU_PHASES = ("bisect_count", "pieces", "tails", "records")


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


def _oracle_run(sc, mode, enc, a, b):
    """The oracle on tags [a, b): (segments, records)."""
    import numpy as np

    import oracle as O

    status, n = O.expand_run(sc, mode=mode, tag_begin=a, tag_end=b, enc=enc)
    assert status == 0
    return int(np.count_nonzero((enc.tags[a:b] & 4) == 0)), n


def cpu_baseline(sc, mode, budget_s=10.0):
    """The FP64 oracle as it stands on a bounded prefix of the same scene:
    once on one thread, then on every host core (one thread per core over
    consecutive tag ranges, the oracle's C code releasing the interpreter
    lock; the ranges' records concatenate in canonical order).  Each run
    takes whole chunks of tags until about budget_s of wall time."""
    import concurrent.futures as F

    import oracle as O

    enc = O.encode(sc)
    O.es_integral(0.0, 0.0, 0.5)  # quadrature nodes initialised before threads start
    n_tags = len(enc.tags)
    step = 20000

    def single():
        # whole passes over the scene's tags, chunk by chunk, until the budget
        w0, c0 = time.time(), time.process_time()
        done = segs = recs = 0
        while done < n_tags or time.time() - w0 < budget_s:
            a = done % n_tags
            b = min(n_tags, a + step)
            s_, r_ = _oracle_run(sc, mode, enc, a, b)
            segs += s_
            recs += r_
            done += b - a
            if done % n_tags == 0 and time.time() - w0 >= budget_s:
                break
        return done, segs, recs, time.time() - w0, time.process_time() - c0

    def multi(threads):
        w0, c0 = time.time(), time.process_time()
        done = segs = recs = 0
        with F.ThreadPoolExecutor(threads) as ex:
            while done < n_tags or time.time() - w0 < budget_s:
                a0 = done % n_tags
                chunks = [(a, min(n_tags, a + step)) for a in range(a0, min(n_tags, a0 + threads * step), step)]
                for s_, r_ in ex.map(lambda ab: _oracle_run(sc, mode, enc, *ab), chunks):
                    segs += s_
                    recs += r_
                done += chunks[-1][1] - a0
                if done % n_tags == 0 and time.time() - w0 >= budget_s:
                    break
        return done, segs, recs, time.time() - w0, time.process_time() - c0

    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    d1, s1, r1, w1, c1 = single()
    dn, sn, rn, wn, cn = multi(cores)
    return {
        "value": sn / wn,
        "unit": "input segs/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{dn / n_tags:g} passes over the scene's {n_tags} tags ({sn} segments, {rn} records), "
                  f"{wn:.1f} s wall / {cn:.1f} s CPU on {cores} threads (one per core, consecutive tag "
                  f"ranges of {step}), FP64",
        "records_per_s": rn / wn,
        "single_thread": {"value": s1 / w1, "unit": "input segs/s", "cores": 1, "records_per_s": r1 / w1,
                          "sample": f"{d1 / n_tags:g} passes ({s1} segments, {r1} records), {w1:.1f} s wall / "
                                    f"{c1:.1f} s CPU"},
        "cpu_model": _cpu_model(),
        "nproc": os.cpu_count(),
    }


# ------------------------------------------------------------------ plain
def work_of(stats, n_tags, n_rec):
    """Algorithmic work of one launch of each phase: flop equivalents
    (WORK x the unit counts of the instrumented run) for the ALU phases,
    bytes for the memory phases."""
    n_slots = stats["pieces"] + n_tags
    curve_pieces = stats["pieces"] - stats["lines"]
    return {
        "bisect_count": stats["trials"] * WORK["trial"],
        "pieces": (curve_pieces * WORK["piece"] + stats["lines"] * WORK["line"] + stats["ranges"] * WORK["range"]
                   + stats["evolutes"] * WORK["evolute"]),
        "tails": stats["joins"] * WORK["join"],
        "records": n_rec * WORK["point"],
        # bytes: tag read + four monoid words written
        "scan_tags": n_tags * 17.0,
        # count read, u64 base written
        "scan_slots": n_tags * 12.0,
        "scan_records": n_slots * 12.0,
        # the write pass writes every piece into the piece list (8 B), reads
        # its kept code (4 B) and each tag's slot count and base (12 B)
        "bisect_write": stats["pieces"] * 12.0 + n_tags * 12.0,
    }


def roofline_of(phase_ms, stats, n_tags, n_rec, mode, names, valu=None):
    """Roofline entry of the dominant phase and the achieved rate of every
    phase: algorithmic work per launch over the average launch time measured
    live.  With VALU counters of the same sources and launch parameters
    (valu: phase -> wave instructions per dispatch), each ALU phase also gets
    its VALU issue rate against one wave instruction per SIMD per clock."""
    work = work_of(stats, n_tags, n_rec)
    dom = max(phase_ms, key=phase_ms.get)
    t_dom = phase_ms[dom] * 1e-3
    if dom in ALU_PHASES:
        achieved = work[dom] / t_dom / 1e12
        roof = {"kernel": dom, "bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_VALU_TFLOPS, "traffic": None,
                "precision": "fp32 points" if dom == "records" else "fp64 decisions"}
    else:
        gbs = work[dom] / t_dom / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": gbs / PEAK_HBM_GBS, "traffic": None}
    roof["algorithmic_work_per_launch"] = work[dom]
    roof["phase_ms"] = phase_ms
    roof["work_counts"] = stats
    roof["work_per_unit"] = WORK
    per = {}
    for n in names:
        t = phase_ms[n] * 1e-3
        if n in ALU_PHASES:
            e = {"TFLOP/s": work[n] / t / 1e12, "frac": work[n] / t / 1e12 / PEAK_VALU_TFLOPS}
            if valu and n in valu:
                rate = valu[n] / t
                e["valu_wave_insts_per_launch"] = valu[n]
                e["valu_issue_frac"] = rate / PEAK_VALU_WAVE_INSTS
        else:
            e = {"GB/s": work[n] / t / 1e9, "frac": work[n] / t / 1e9 / PEAK_HBM_GBS}
        per[n] = e
    roof["per_kernel"] = per
    if valu and dom in valu:
        roof["valu_issue"] = {"achieved": valu[dom] / t_dom, "peak": PEAK_VALU_WAVE_INSTS, "unit": "wave-insts/s",
                              "frac": valu[dom] / t_dom / PEAK_VALU_WAVE_INSTS}
    return roof


TUNE_CACHE = os.path.join(ROOT, "paper_2405_00127_amd", "tuning.json")


def time_steps(ctx, scene, tol, mode, buf, cnt, stream, steps, warmup, torch):
    """Average ms of one whole-pipeline step (sx_expand_async, inputs resident
    in HBM), host clock around `steps` launches bracketed by device syncs."""
    def step():
        ctx.expand_async(scene, buf.data_ptr(), buf.numel(), cnt.data_ptr(), tol, mode, stream=stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps


def phase_times(ctx, scene, tol, mode, buf, stream, steps, B, torch):
    """Average ms of each pipeline phase: HIP events recorded on the stream the
    phase kernels are launched on, around each phase launch."""
    names = B.PHASE_NAMES
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in names]
           for _ in range(steps)]
    for k in range(steps):
        for p in range(len(names)):
            evs[k][p][0].record(stream)
            ctx.run_phase(scene, p, tol, mode, buf.data_ptr(), buf.numel(), stream=stream)
            evs[k][p][1].record(stream)
    torch.cuda.synchronize()
    return {names[p]: sum(evs[k][p][0].elapsed_time(evs[k][p][1]) for k in range(steps)) / steps
            for p in range(len(names))}


def plain(args, ctx, B, S, torch, np):
    mode = S.OUT_LINES if args.mode == "lines" else S.OUT_ARCS
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    log("bench: generating the map scene")
    sc = S.scene_map(2, args.segments, args.paths, 0.25, mode)
    if args.fill_scene:
        sc = S.with_fills(sc)
    if args.dashed_scene:
        sc = S.with_dashes(sc, seed=4, lo=0.5, hi=12.0)
    n_seg = sc.n_segments()
    scene = ctx.encode(sc, stream=stream)
    dash_ms = []
    if args.dashed_scene:
        # the dash passes run at encoding: encode twice more for their timings
        dash_ms.append(scene.dash_ms())
        for _ in range(2):
            scene.release()
            scene = ctx.encode(sc, stream=stream)
            dash_ms.append(scene.dash_ms())
        log(f"bench: dash passes {dash_ms} ms, {scene.n_tags} dashed tags")
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
        tune_info["source"] = "command line"
    elif not args.no_tune:
        from paper_2405_00127_amd import autotune as AT

        log("bench: launch parameters from the autotuner" + (" (retuning)" if args.retune else " (cache)"))
        _, times = AT.tune(ctx, scene, tol, mode, buf.data_ptr(), buf.numel(), cnt.data_ptr(), stream,
                           cache_path=args.tune_cache, use_cache=not args.retune, counts=cnt)
        tune_info = {"source": "autotuner, timed now" if times else f"autotuner cache {os.path.relpath(args.tune_cache, ROOT)}",
                     "candidates_ms": times}
    tune_info["chosen"] = ctx.get_tuning()
    log(f"bench: tuning {tune_info['chosen']}")

    ms = time_steps(ctx, scene, tol, mode, buf, cnt, stream, args.steps, args.warmup, torch)
    assert int(cnt[0].item()) == n_rec and int(cnt[1].item()) == 0
    log(f"bench: plain {ms:.3f} ms/step")
    names = B.PHASE_NAMES
    phase_ms = phase_times(ctx, scene, tol, mode, buf, stream, args.steps, B, torch)
    log("bench: phases " + ", ".join(f"{n} {phase_ms[n]:.3f} ms" for n in names))
    stats = ctx.piece_stats(scene, tol, mode, stream=stream)
    log(f"bench: work {stats}")

    n_tags = scene.n_tags
    counters = (None if (args.fill_scene or args.dashed_scene or args.density != "approx")
                else measured_counters(args.mode, tune_info["chosen"]))
    roof = roofline_of(phase_ms, stats, n_tags, n_rec, mode, names,
                       valu=counters["valu"] if counters else None)
    if counters and roof["kernel"] in counters["traffic"]:
        roof["traffic"] = counters["traffic"][roof["kernel"]]
        roof["traffic_source"] = counters["source"]
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
                        + ("dash pattern on every stroke, " if args.dashed_scene else "")
                        + ("exact density with Newton-refined inverse, " if args.density != "approx" else "")
                        + f"plain per-scene expansion, {args.mode}, tol 0.25 px",
            "segments": n_seg, "tags": n_tags, "records": n_rec, "output": args.mode, "tolerance": tol,
        },
        "output_records_per_s": n_rec / (ms * 1e-3),
        "roofline": roof,
        "tuning": tune_info,
    }
    if dash_ms:
        out["dash_ms"] = dash_ms
    del buf
    return out, sc, mode


def legs(args, ctx, B, S, torch, np):
    """The other single-scene configurations, with the plain leg's launch
    parameters: the 1k-cubic scene (lines; also replayed as a captured HIP
    graph, since a scene this small is bound by launch overhead), the map
    scene with arc output, the 100k-cubic stress scene (arcs, 0.1 px), the
    map scene with lines counted and placed by the exact density integral,
    and the map scene with a dash pattern on every stroke (dash passes timed
    at encoding, then the expansion of the dashed scene)."""
    stream = torch.cuda.current_stream()
    dev = torch.device("cuda:0")
    res = {}
    # the exact-density mode (Section 4.2's Newton-refined inverse) runs on a
    # context of its own, with the same launch parameters
    ctx_n = B.Context(0, density=B.DENSITY_NEWTON)
    ctx_n.set_tuning(**ctx.get_tuning())
    for name, make, c in (("c1_lines", lambda: S.scene_c1(1), ctx),
                          ("map1M_arcs", lambda: S.scene_map(2, args.segments, args.paths, 0.25, S.OUT_ARCS), ctx),
                          ("stress100k_arcs", lambda: S.scene_c3(3), ctx),
                          ("map1M_lines_exact_density",
                           lambda: S.scene_map(2, args.segments, args.paths, 0.25, S.OUT_LINES), ctx_n),
                          ("map1M_dashed_lines",
                           lambda: S.with_dashes(S.scene_map(2, args.segments, args.paths, 0.25, S.OUT_LINES),
                                                 seed=4, lo=0.5, hi=12.0), ctx)):
        ctx_saved, ctx = ctx, c
        sc = make()
        mode = sc.output_mode
        scene = ctx.encode(sc, stream=stream)
        tol = sc.tolerance
        _, n_rec, buf = ctx.expand(scene, tol, mode, stream=stream)
        cnt = torch.zeros(2, dtype=torch.int64, device=dev)
        steps = args.steps * (10 if name == "c1_lines" else 1)
        ms = time_steps(ctx, scene, tol, mode, buf, cnt, stream, steps, args.warmup, torch)
        assert int(cnt[0].item()) == n_rec and int(cnt[1].item()) == 0
        phase_ms = phase_times(ctx, scene, tol, mode, buf, stream, args.steps, B, torch)
        stats = ctx.piece_stats(scene, tol, mode, stream=stream)
        roof = roofline_of(phase_ms, stats, scene.n_tags, n_rec, mode, B.PHASE_NAMES)
        n_seg = sc.n_segments()
        r = {"workload": sc.name, "segments": n_seg, "tags": scene.n_tags, "records": n_rec,
             "output": "arcs" if mode == S.OUT_ARCS else "lines", "tolerance": tol,
             "ms_per_step": ms, "segs_per_s": n_seg / (ms * 1e-3), "records_per_s": n_rec / (ms * 1e-3),
             "phase_ms": phase_ms,
             "roofline": {k: roof[k] for k in ("kernel", "bound", "achieved", "peak", "unit", "frac")}}
        if sc.dashes is not None:
            # the dash passes run once, at encoding (device time measured there);
            # the oracle's dashing of the same scene on one host core beside it
            import oracle as O

            t0 = time.perf_counter()
            O.encode_dashed(sc)
            r["dash_ms"] = scene.dash_ms()
            r["dashed_tags"] = scene.n_tags
            r["oracle_dash_ms_one_core"] = (time.perf_counter() - t0) * 1e3
        if name == "c1_lines":
            s2 = torch.cuda.Stream()
            with torch.cuda.stream(s2):
                ctx.expand_async(scene, buf.data_ptr(), buf.numel(), cnt.data_ptr(), tol, mode, stream=s2)
            s2.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s2):
                ctx.expand_async(scene, buf.data_ptr(), buf.numel(), cnt.data_ptr(), tol, mode, stream=s2)
            s2.synchronize()
            for _ in range(3):
                g.replay()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                g.replay()
            torch.cuda.synchronize()
            gms = (time.perf_counter() - t0) * 1e3 / steps
            assert int(cnt[0].item()) == n_rec
            r["graph_ms_per_step"] = gms
            r["graph_segs_per_s"] = n_seg / (gms * 1e-3)
            del g
        log(f"bench: leg {name}: {ms:.3f} ms/step, {n_rec} records")
        res[name] = r
        scene.release()
        del buf
        ctx = ctx_saved
    ctx_n.close()
    return res


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
    ms = time_steps(ctx, scene, tol, mode, buf, cnt, stream, args.steps, args.warmup, torch)
    assert int(cnt[0].item()) == n_rec and int(cnt[1].item()) == 0
    names = B.PHASE_NAMES
    phase_ms = phase_times(ctx, scene, tol, mode, buf, stream, args.steps, B, torch)
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
    # the batch's own launch parameters: the autotuner on the arena (cached
    # per size bucket); the per-scene loop runs with the same ones
    from paper_2405_00127_amd import autotune as AT

    plain_tuning = ctx.get_tuning()
    bcnt = torch.zeros(2, dtype=torch.int64, device=dev)
    _, btimes = AT.tune(ctx, batch.arena(), tol, mode, bout.data_ptr(), bout.numel(), bcnt.data_ptr(), stream,
                        cache_path=args.tune_cache, use_cache=not args.retune, counts=bcnt)
    batch_tuning = ctx.get_tuning()
    log(f"bench: batch tuning {batch_tuning}" + (" (timed now)" if btimes else " (cache)"))
    with torch.cuda.stream(stream):  # the workspaces of the loop's scenes, for the batch's chunk size
        for i, s in enumerate(scenes):
            ctx.expand_into(s, buf.data_ptr() + int(starts[i]) * rec, int(counts[i]) * rec, tol, mode, stream)

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
    ctx.set_tuning(**plain_tuning)
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
        "tuning": {"chosen": batch_tuning, "candidates_ms": btimes},
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
    """Hash of the HIP sources without comments and blank space, and of the
    compiler flags they are built with: counter readings are tied to the
    code they were taken on."""
    import hashlib
    import re

    from paper_2405_00127_amd import build as PB

    h = hashlib.sha256()
    h.update(" ".join(PB.FLAGS).encode() + b"\0")
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


def measured_counters(mode: str, tuning: dict):
    """HBM bytes and VALU wave instructions per launch of each phase from the
    committed rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a
    plain copy's reading; SQ_INSTS_VALU), or None when the summary is missing
    or was taken on other kernel sources or launch parameters."""
    path = os.path.join(ROOT, "profiles", f"counters_map1M_{mode}.json")
    try:
        with open(path, "r", encoding="utf-8") as f:
            data = json.load(f)
    except (OSError, ValueError):
        return None
    if data.get("kernel_source_hash") != kernel_source_hash():
        return None
    if {k: int(v) for k, v in data.get("tuning", {}).items()} != {k: int(v) for k, v in tuning.items()}:
        return None
    return {"traffic": {k: v["bytes_per_launch"] for k, v in data.get("kernels", {}).items()},
            "valu": {k: v["valu_insts"] for k, v in data.get("valu", {}).items()},
            "source": os.path.relpath(path, ROOT)}


def phase_of_kernel(name: str):
    """Pipeline phase of a rocprofv3 kernel name (None for other kernels and
    for the launch variants with work counters, which run only to count)."""
    import re

    simple = (("scan_tags_kernel", "scan_tags"), ("scan_counts_kernel", "scan_slots"),
              ("scan_counts_dev_kernel", "scan_records"), ("finish_kernel", "finish"))
    for key, phase in simple:
        if f"sx::{key}(" in name:
            return phase
    if re.search(r"sx::record_kernel(<(true|false)>)?\(", name):
        return "records"
    m = re.search(r"sx::bisect_kernel<(true|false), (true|false), \d+>", name)
    if m:
        return None if m.group(2) == "true" else ("bisect_write" if m.group(1) == "true" else "bisect_count")
    m = re.search(r"sx::slot_kernel<\d+, (true|false)(, (true|false))?>", name)
    if m:
        return None if m.group(1) == "true" else "pieces"
    m = re.search(r"sx::tail_kernel<(true|false)>", name)
    if m:
        return None if m.group(1) == "true" else "tails"
    return None


def summarize_counters(fetch_db: str, write_db: str, valu_db: str, probe_mb: int, mode: str, tuning: dict,
                       commands) -> dict:
    """Per-launch HBM bytes of each phase from two rocprofv3 --pmc databases
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch), each scaled by what the same
    counter reads for the plain copy of probe_mb MiB that --copy-probe runs
    (the largest runtime copy kernel of the run), and the VALU counters of a
    third database (summarize_valu)."""
    import sqlite3

    probe = float(probe_mb << 20)
    out = {"kernel_source_hash": kernel_source_hash(), "workload": f"map1M_{mode}", "tuning": tuning,
           "commands": list(commands), "calibration": {"probe_bytes": probe}, "kernels": {}}
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
    out["valu"] = summarize_valu(valu_db)
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
        # offline: bench.py --summarize-counters FETCH_DB WRITE_DB VALU_DB PROBE_MB MODE TUNING_JSON [COMMAND ...]
        fetch_db, write_db, valu_db, probe_mb, mode, tuning = sys.argv[2:8]
        res = summarize_counters(fetch_db, write_db, valu_db, int(probe_mb), mode, json.loads(tuning), sys.argv[8:])
        path = os.path.join(ROOT, "profiles", f"counters_map1M_{mode}.json")
        with open(path, "w", encoding="utf-8") as f:
            json.dump(res, f, indent=1)
        print(json.dumps({"kernels": res["kernels"], "valu": res["valu"]}, indent=1))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["lines", "arcs"], default="lines")
    ap.add_argument("--segments", type=int, default=1_000_000)
    ap.add_argument("--paths", type=int, default=10_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=10.0)
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-parameter autotuner")
    ap.add_argument("--retune", action="store_true", help="time the autotuner's candidates instead of its cache")
    ap.add_argument("--tune-cache", default=TUNE_CACHE, help="autotuner cache file")
    ap.add_argument("--no-legs", action="store_true", help="skip the 1k-cubic, map-arcs and stress legs")
    ap.add_argument("--piece-waves", type=int, default=None)
    ap.add_argument("--chunk-k", type=int, default=None)
    ap.add_argument("--bisect-range", type=int, default=None)
    ap.add_argument("--bisect-waves", type=int, default=None)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-fill", action="store_true", help="skip the fill leg (the map scene filled)")
    ap.add_argument("--fill-scene", action="store_true",
                    help="time the map scene with every path filled in the main leg (for profiling the fill)")
    ap.add_argument("--dashed-scene", action="store_true",
                    help="time the map scene with a dash pattern on every stroke in the main leg (for profiling)")
    ap.add_argument("--density", choices=["approx", "newton"], default="approx",
                    help="main leg's density mode (newton: exact integral, Newton-refined inverse; for profiling)")
    ap.add_argument("--batch-scenes", type=int, default=256)
    ap.add_argument("--batch-steps", type=int, default=10)
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--pool", type=int, default=64)
    ap.add_argument("--qps", type=float, nargs="*", default=[100.0, 200.0, 500.0, 1000.0, 2000.0, 5000.0])
    ap.add_argument("--serve-seconds", type=float, default=10.0)
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
    ctx = B.Context(0, density=B.DENSITY_NEWTON if args.density == "newton" else B.DENSITY_APPROX)
    if args.copy_probe:
        n = args.copy_probe << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    out, sc, mode = plain(args, ctx, B, S, torch, np)
    if not args.no_legs:
        out["legs"] = legs(args, ctx, B, S, torch, np)
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
            out["fill"]["cpu_baseline"] = cpu_baseline(fill_sc, mode, min(args.cpu_budget, 4.0))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
