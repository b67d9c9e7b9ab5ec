"""Continuous-batching expansion server (one GPU, one host thread).

Requests name already encoded, device-resident scenes.  The server keeps a
small ring of *slots*; a slot owns a batch arena, an output arena, per-scene
offsets and status words, its own HIP stream (default priority) and a
completion event.  The loop

  1. admits arrived requests into the pending queue;
  2. whenever a slot is free, takes pending requests in arrival order while
     the slot's memory budget allows (segments into the batch arena, a
     predicted record count into the output arena), gathers them into the
     slot's arena and launches the batched pipeline on the slot's stream --
     so requests that arrive while other batches run on the GPU join the next
     free slot and their work overlaps on the device.  A request taken alone
     runs as a plain expansion of its own scene (no gather), unless another
     slot is expanding that scene: a scene's own workspace serves one
     expansion at a time;
  3. polls in-flight slots; a finished slot reports each request's record
     range and frees its memory.

The record count of a request is unknown until its count pass ran, so the
admission predicts it from the running maximum of records per input segment
seen so far (times a margin).  A batch whose total still exceeds its output
arena emits nothing (the library guarantees it); the server then grows that
arena and re-runs the batch, which only adds latency.

This module is host logic only: every step of the expansion runs in the HIP
kernels behind the C ABI.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Deque, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    scene: object          # binding.Scene (device-resident)
    n_segments: int
    arrival: float         # host clock (s) at which the request arrived
    admitted: float = 0.0
    done: float = 0.0
    slot: int = -1
    first: int = 0         # record range in the slot's output arena
    count: int = 0


class _Slot:
    def __init__(self, ctx, index: int, tolerance: float, mode: int, seg_budget: int, rec_budget: int):
        import torch

        from . import binding as B

        self.index = index
        self.ctx = ctx
        self.tol = tolerance
        self.mode = mode
        self.batch = B.Batch(ctx)
        self.stream = torch.cuda.Stream(device=ctx.device)  # default priority
        self.event = torch.cuda.Event()
        self.rec = B.RECORD_BYTES[mode]
        self.seg_budget = seg_budget
        self.rec_budget = rec_budget
        dev = f"cuda:{ctx.device}"
        self.out = torch.empty(rec_budget * self.rec, dtype=torch.uint8, device=dev)
        self.offs = torch.zeros(1, dtype=torch.int64, device=dev)
        self.status = torch.zeros(2, dtype=torch.int64, device=dev)
        self.host = torch.zeros(2, dtype=torch.int64).pin_memory()
        self.host_offs = torch.zeros(1, dtype=torch.int64).pin_memory()
        self.reqs: List[Request] = []
        self.single = None  # the scene of a one-request batch (run as a plain expansion)
        self.busy = False
        self.reruns = 0

    def launch(self, reqs: List[Request], alone_ok: bool = True):
        """Run ``reqs`` on the slot's stream.  ``alone_ok``: a single request
        may run as a plain expansion of its own scene, which uses the scene's
        own workspace -- only allowed when no other slot is expanding that
        scene."""
        import torch

        self.reqs = reqs
        n = len(reqs)
        dev = self.out.device
        if self.offs.numel() < n + 1:
            self.offs = torch.zeros(n + 1, dtype=torch.int64, device=dev)
            self.host_offs = torch.zeros(n + 1, dtype=torch.int64).pin_memory()
        # a request alone runs as a plain expansion of its own scene (no
        # gather into the arena, no per-scene offsets)
        self.single = reqs[0].scene if (n == 1 and alone_ok) else None
        if self.single is None:
            self.batch.set([r.scene for r in reqs], stream=self.stream)
        self._run()
        self.busy = True

    def _run(self):
        n = len(self.reqs)
        if self.single is not None:
            self.ctx.expand_async(self.single, self.out.data_ptr(), self.out.numel(), self.status.data_ptr(),
                                  self.tol, self.mode, stream=self.stream)
        else:
            self.batch.expand_async(self.tol, self.mode, self.out.data_ptr(), self.out.numel(),
                                    self.offs.data_ptr(), self.status.data_ptr(), stream=self.stream)
        with __import__("torch").cuda.stream(self.stream):
            self.host.copy_(self.status, non_blocking=True)
            if self.single is None:
                self.host_offs[: n + 1].copy_(self.offs[: n + 1], non_blocking=True)
        self.event.record(self.stream)

    def poll(self) -> bool:
        """True once the slot's batch is complete (re-running it first if its
        output or item workspace was too small)."""
        import torch

        if not self.busy or not self.event.query():
            return False
        total, need = int(self.host[0]), int(self.host[1])
        if need or total > self.rec_budget:
            # grow what was too small and run the batch again
            self.reruns += 1
            if need:
                from . import binding as B

                # a synchronous expansion resizes the item workspace
                scene = self.single if self.single is not None else self.batch.arena()
                probe = torch.empty(16, dtype=torch.uint8, device=self.out.device)
                try:
                    total = self.ctx.expand_into(scene, probe.data_ptr(), 0, self.tol, self.mode, self.stream)
                except B.StrokexError as e:
                    if e.code != B.SX_ETOOSMALL:
                        raise
                    total = e.required
            if total > self.rec_budget:
                self.rec_budget = int(total * 1.25) + 1
                self.out = torch.empty(self.rec_budget * self.rec, dtype=torch.uint8, device=self.out.device)
            self._run()
            return False
        if self.single is not None:
            offs = np.array([0, total], dtype=np.int64)
        else:
            offs = self.host_offs[: len(self.reqs) + 1].numpy()
        for i, r in enumerate(self.reqs):
            r.first = int(offs[i])
            r.count = int(offs[i + 1] - offs[i])
            r.slot = self.index
        self.busy = False
        return True

    def records(self, r: Request):
        """Device float32 view [count, 5|6] of a finished request's records
        (valid until the slot runs its next batch)."""
        a = self.out[r.first * self.rec:(r.first + r.count) * self.rec]
        return a.view(__import__("torch").float32).view(-1, self.rec // 4)

    def destroy(self):
        self.batch.destroy()


class Server:
    """Continuous batching over ``n_slots`` slots.

    seg_budget   input segments one slot's batch may hold (batch arena);
    rec_budget   output records one slot's arena holds initially;
    max_batch    requests per batch;
    rec_margin   factor on the running max records/segment for admission;
    on_done      optional callable(request, records) run when a request
                 finishes, before its slot takes new work: ``records`` is a
                 device float32 [count, 5|6] view, valid only during the call.
    """

    def __init__(self, ctx, tolerance: float, mode: int, n_slots: int = 3, seg_budget: int = 4_000_000,
                 rec_budget: int = 60_000_000, max_batch: int = 256, rec_margin: float = 1.5, on_done=None):
        self.ctx = ctx
        self.on_done = on_done
        self.tol = tolerance
        self.mode = mode
        self.slots = [_Slot(ctx, i, tolerance, mode, seg_budget, rec_budget) for i in range(n_slots)]
        self.max_batch = max_batch
        self.rec_margin = rec_margin
        self.rec_per_seg = 0.0
        self.pending: Deque[Request] = collections.deque()
        self.done: List[Request] = []
        self.batches = 0

    def submit(self, req: Request):
        self.pending.append(req)

    def _predict(self, r: Request) -> int:
        rps = self.rec_per_seg if self.rec_per_seg > 0 else 40.0
        return int(r.n_segments * rps * self.rec_margin) + 64

    def step(self, now: float) -> int:
        """One scheduler pass: retire finished slots, fill free ones.
        Returns the number of requests completed in this pass."""
        finished = 0
        for sl in self.slots:
            if sl.busy and sl.poll():
                t = time.perf_counter()
                for r in sl.reqs:
                    r.done = t
                    if r.n_segments:
                        self.rec_per_seg = max(self.rec_per_seg, r.count / r.n_segments)
                    if self.on_done is not None:
                        self.on_done(r, sl.records(r))
                    self.done.append(r)
                    finished += 1
                sl.reqs = []
        for sl in self.slots:
            if sl.busy or not self.pending:
                continue
            take: List[Request] = []
            segs = 0
            recs = 0
            while self.pending and len(take) < self.max_batch:
                r = self.pending[0]
                p = self._predict(r)
                fits = (segs + r.n_segments <= sl.seg_budget and recs + p <= sl.rec_budget)
                if take and not fits:
                    break
                # a request larger than a whole slot still runs alone (the
                # slot grows for it)
                self.pending.popleft()
                r.admitted = now
                take.append(r)
                segs += r.n_segments
                recs += p
            # a scene's own workspace serves one plain expansion at a time
            alone_ok = len(take) == 1 and not any(
                o is not sl and o.busy and o.single is take[0].scene for o in self.slots)
            sl.launch(take, alone_ok)
            self.batches += 1
        return finished

    def busy(self) -> bool:
        return bool(self.pending) or any(sl.busy for sl in self.slots)

    def close(self):
        for sl in self.slots:
            sl.destroy()


def poisson_arrivals(seed: int, qps: float, n: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / qps, n))


def run_load(ctx, pool, pool_segments, qps: float, n_requests: int, tolerance: float, mode: int, seed: int = 5,
             max_seconds: float = 10.0, server_kwargs: Optional[dict] = None,
             server: Optional["Server"] = None) -> Dict[str, float]:
    """Drive a server with Poisson arrivals at ``qps`` over requests drawn
    uniformly from ``pool`` (encoded scenes).  ``server``: an existing idle
    server to reuse (its slots keep the arenas and workspaces earlier loads
    grew; it is left open), else a new one is made and closed.  Returns
    throughput and latency percentiles (ms)."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    arr = poisson_arrivals(seed, qps, n_requests)
    picks = rng.integers(0, len(pool), n_requests)
    own = server is None
    srv = Server(ctx, tolerance, mode, **(server_kwargs or {})) if own else server
    if not own:
        if srv.busy():
            raise ValueError("run_load needs an idle server")
        srv.done = []
        srv.batches = 0
        for sl in srv.slots:
            sl.reruns = 0
    t0 = time.perf_counter()
    i = 0
    while True:
        now = time.perf_counter() - t0
        while i < n_requests and arr[i] <= now and now < max_seconds:
            k = int(picks[i])
            srv.submit(Request(i, pool[k], int(pool_segments[k]), t0 + arr[i]))
            i += 1
        srv.step(time.perf_counter())
        if (i >= n_requests or now >= max_seconds) and not srv.busy():
            break
    t_end = time.perf_counter()
    lat = np.array([(r.done - r.arrival) * 1e3 for r in srv.done])
    segs = sum(r.n_segments for r in srv.done)
    recs = sum(r.count for r in srv.done)
    span = max(t_end - t0, 1e-9)
    out = {
        "qps": qps,
        "requests": len(srv.done),
        "segs_per_s": segs / span,
        "records_per_s": recs / span,
        "p50_ms": float(np.percentile(lat, 50)) if len(lat) else float("nan"),
        "p99_ms": float(np.percentile(lat, 99)) if len(lat) else float("nan"),
        "batches": srv.batches,
        "reruns": sum(sl.reruns for sl in srv.slots),
    }
    if own:
        srv.close()
    return out


def run_serial(ctx, pool, pool_segments, qps: float, n_requests: int, tolerance: float, mode: int, seed: int = 5,
               max_seconds: float = 10.0) -> Dict[str, float]:
    """Baseline: serial FIFO, one plain expansion per request on one stream."""
    import torch

    rng = np.random.Generator(np.random.PCG64(seed + 1))
    arr = poisson_arrivals(seed, qps, n_requests)
    picks = rng.integers(0, len(pool), n_requests)
    from . import binding as B

    stream = torch.cuda.Stream(device=ctx.device)
    rec = B.RECORD_BYTES[mode]
    cap = 60_000_000
    out = torch.empty(cap * rec, dtype=torch.uint8, device=f"cuda:{ctx.device}")
    cnt = torch.zeros(2, dtype=torch.int64, device=f"cuda:{ctx.device}")
    ev = torch.cuda.Event()
    t0 = time.perf_counter()
    lat = []
    segs = 0
    i = 0
    while i < n_requests:
        now = time.perf_counter() - t0
        if now >= max_seconds:
            break
        if arr[i] > now:
            continue
        k = int(picks[i])
        ctx.expand_async(pool[k], out.data_ptr(), out.numel(), cnt.data_ptr(), tolerance, mode, stream=stream)
        ev.record(stream)
        ev.synchronize()
        lat.append((time.perf_counter() - (t0 + arr[i])) * 1e3)
        segs += int(pool_segments[k])
        i += 1
    span = max(time.perf_counter() - t0, 1e-9)
    lat = np.array(lat)
    return {
        "qps": qps,
        "requests": len(lat),
        "segs_per_s": segs / span,
        "p50_ms": float(np.percentile(lat, 50)) if len(lat) else float("nan"),
        "p99_ms": float(np.percentile(lat, 99)) if len(lat) else float("nan"),
    }
