#!/usr/bin/env python
"""Benchmark of GPU stroke expansion on one MI355X.

Headline: input path segments expanded per second at 0.25 px tolerance on
the map/CAD-shaped scene (10,000 paths, 1,000,000 segments: 60% lines, 15%
quads, 25% cubics, mixed joins/caps, lognormal half-widths), line output.
One step = the whole hot path over the scene already resident in HBM: tag
monoid scan, per-segment counts, count scan, emission.

Prints one JSON line (see the design doc for the roofline model).
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
# Algorithmic FP32 work per output record of the emit kernel (one new
# outline point per record):
#   spiral position: 4-node Gauss-Legendre, 4 x (phase 4 + sincos 36 + 2 FMA 4) = 176
#   normal: phase 4 + sincos 36 = 40; offset + rotation 10; record write 0
#   point placement (inverse of the density integral, lines): ~24 + asin 30 = 54
#   arc mode replaces placement by the sweep: 2 phases 8 + sin 18 + chord 6 = 32
FLOPS_PER_RECORD = {0: 280.0, 1: 258.0}
RECORD_BYTES = {0: 20, 1: 24}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(sc, mode, budget_s=12.0):
    """The FP64 oracle (single thread, as it stands) on a bounded prefix of the
    same scene: whole paths, grown until ~budget_s of CPU time."""
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


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--mode", choices=["lines", "arcs"], default="lines")
    ap.add_argument("--segments", type=int, default=1_000_000)
    ap.add_argument("--paths", type=int, default=10_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {args.gpus}); "
              "stroke expansion of independent scenes would shard by scene, see DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2405_00127_amd import binding as B
    from paper_2405_00127_amd import build as PB
    from paper_2405_00127_amd import scenes as S

    if not os.path.exists(B.LIB_PATH):
        PB.build()
    mode = S.OUT_LINES if args.mode == "lines" else S.OUT_ARCS
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    log("bench: generating scene")
    sc = S.scene_map(2, args.segments, args.paths, 0.25, mode)
    n_seg = sc.n_segments()
    ctx = B.Context(0)
    log("bench: encoding")
    scene = ctx.encode(sc, stream=stream)
    tol = sc.tolerance
    # size the output once (not timed)
    recs, n_rec, buf = ctx.expand(scene, tol, mode, stream=stream)
    cnt = torch.zeros(2, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    log(f"bench: {n_seg} segments, {scene.n_tags} tags -> {n_rec} records")

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
    log(f"bench: {ms:.3f} ms/step")

    # per-kernel times: HIP events on the launching stream around each phase
    nph = 4
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(nph)]
           for _ in range(args.steps)]
    for k in range(args.steps):
        for p in range(nph):
            evs[k][p][0].record(stream)
            ctx.run_phase(scene, p, tol, mode, buf.data_ptr(), buf.numel(), stream=stream)
            evs[k][p][1].record(stream)
    torch.cuda.synchronize()
    phase_ms = [sum(evs[k][p][0].elapsed_time(evs[k][p][1]) for k in range(args.steps)) / args.steps
                for p in range(nph)]
    names = B.PHASE_NAMES
    dom = int(np.argmax(phase_ms))
    log("bench: phases " + ", ".join(f"{names[p]} {phase_ms[p]:.3f} ms" for p in range(nph)))

    n_tags = scene.n_tags
    if names[dom] == "records":
        flops = n_rec * FLOPS_PER_RECORD[mode]
        achieved = flops / (phase_ms[dom] * 1e-3) / 1e12
        roof = {"kernel": "records", "bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                "units_per_launch": {"records": n_rec}, "flops_per_record": FLOPS_PER_RECORD[mode]}
    elif names[dom] in ("scan_tags", "scan_counts"):
        per = 17 if names[dom] == "scan_tags" else 12
        gbs = n_tags * per / (phase_ms[dom] * 1e-3) / 1e9
        roof = {"kernel": names[dom], "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": gbs / PEAK_HBM_GBS, "traffic": None}
    else:
        # the count kernel does the emit kernel's per-piece decisions without
        # the per-point work; its algorithmic work is charged per record too
        flops = n_rec * FLOPS_PER_RECORD[mode]
        achieved = flops / (phase_ms[dom] * 1e-3) / 1e12
        roof = {"kernel": "pieces", "bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None}
    roof["phase_ms"] = {names[p]: phase_ms[p] for p in range(nph)}
    roof["emit_hbm_GBps"] = (n_rec * RECORD_BYTES[mode] + n_tags * 48) / (phase_ms[3] * 1e-3) / 1e9

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
                        f"plain per-scene expansion, {args.mode}, tol 0.25 px",
            "segments": n_seg, "tags": n_tags, "records": n_rec, "output": args.mode, "tolerance": tol,
        },
        "output_records_per_s": n_rec / (ms * 1e-3),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(sc, mode, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
