"""Batched expansion (many scenes, one pipeline) through the C ABI.

A scene's outline must be the same alone and in a batch, bit for bit (the
arena is a concatenation; every per-segment computation sees the same
inputs), with the scene's own path indices; the batched launch must survive
HIP graph capture and replay."""
import sys

import numpy as np
import pytest

from paper_2405_00127_amd import scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2405_00127_amd import binding as B
    from paper_2405_00127_amd import build as PB

    if not __import__("os").path.exists(B.LIB_PATH):
        PB.build()
    torch.cuda.set_device(0)
    c = B.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mixed_scenes(mode):
    empty = S.SceneBuilder().build(S.make_styles([1.0], S.JOIN_ROUND, S.CAP_BUTT))
    return [
        S.scene_c1(1).subset(range(7)),
        S.scene_map(11, 5000, 40, 0.25, mode),
        empty,
        S.scene_c3(3, n_cubics=120),
        S.scene_map(12, 300, 3, 0.25, mode),
        S.single_path_scene([S.MOVE, S.LINE], [(10.0, 10.0), (40.0, 12.0)], 3.0, S.JOIN_MITER, S.CAP_SQUARE,
                            output_mode=mode),
        S.scene_map(14, 20000, 150, 0.25, mode),
        # fills: a filled map scene, and half fills under a shear
        S.with_fills(S.scene_map(15, 4000, 30, 0.25, mode)),
        S.with_fills(S.scene_c1(1, output_mode=mode).subset(range(5)), 0.5, seed=2,
                     xform=[1.0, 0.2, 0.5, 0.9, 10.0, -5.0]),
        # dashed scenes are ordinary scenes once encoded
        S.with_dashes(S.scene_map(16, 3000, 20, 0.25, mode), seed=5, lo=0.5, hi=12.0),
        S.with_dashes(S.scene_c1(1, output_mode=mode).subset(range(4)), seed=6),
    ]


def _alone(ctx, scene, tol, mode):
    from paper_2405_00127_amd import binding as B

    recs, n, _ = ctx.expand(scene, tol, mode)
    return B.records_to_numpy(recs, mode).copy() if n else np.zeros(0, B.LINE_DTYPE if mode == 0 else B.ARC_DTYPE)


def _slices(buf, offs, mode):
    from paper_2405_00127_amd import binding as B

    rec = B.RECORD_BYTES[mode]
    total = int(offs[-1])
    allr = B.records_to_numpy(buf[: total * rec].view(__import__("torch").float32).view(-1, rec // 4), mode) \
        if total else np.zeros(0, B.LINE_DTYPE if mode == 0 else B.ARC_DTYPE)
    return [allr[int(offs[i]):int(offs[i + 1])] for i in range(len(offs) - 1)]


@pytest.mark.parametrize("mode", [S.OUT_LINES, S.OUT_ARCS])
def test_batch_equals_scenes_alone(ctx, mode):
    import torch

    from paper_2405_00127_amd import binding as B

    tol = 0.25
    scs = _mixed_scenes(mode)
    _say("batch vs alone, mode", mode, [s.name for s in scs])
    scenes = [ctx.encode(sc) for sc in scs]
    alone = [_alone(ctx, s, tol, mode) for s in scenes]
    batch = B.Batch(ctx)
    batch.set(scenes)
    out, offs, status = batch.prepare(tol, mode)
    batch.expand_async(tol, mode, out.data_ptr(), out.numel(), offs.data_ptr(), status.data_ptr())
    torch.cuda.synchronize()
    o = offs.cpu().numpy()
    assert int(status[1]) == 0 and int(status[0]) == o[-1] == sum(len(a) for a in alone)
    for i, (got, ref) in enumerate(zip(_slices(out, o, mode), alone)):
        assert len(got) == len(ref), i
        assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), i
    batch.destroy()


def test_batch_graph_replay_and_reuse(ctx):
    """Capture the batched launch in a graph, replay it three times with eager
    work in between, then reuse the batch for a smaller set of scenes."""
    import torch

    from paper_2405_00127_amd import binding as B

    tol, mode = 0.25, S.OUT_LINES
    scs = [S.scene_map(20 + i, n, max(1, n // 100), tol, mode) for i, n in enumerate([150, 9000, 40, 30000, 2500])]
    _say("batch graph replay", [s.n_segments() for s in scs])
    scenes = [ctx.encode(sc) for sc in scs]
    alone = [_alone(ctx, s, tol, mode) for s in scenes]
    batch = B.Batch(ctx)
    batch.set(scenes)
    out, offs, status = batch.prepare(tol, mode)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        # warm up on the capture stream, then capture
        batch.expand_async(tol, mode, out.data_ptr(), out.numel(), offs.data_ptr(), status.data_ptr(), stream=side)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        batch.expand_async(tol, mode, out.data_ptr(), out.numel(), offs.data_ptr(), status.data_ptr(), stream=side)
    for rep in range(3):
        out.zero_()
        offs.zero_()
        junk = torch.randn(1 << 16, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        o = offs.cpu().numpy()
        assert int(status[1]) == 0, rep
        for i, (got, ref) in enumerate(zip(_slices(out, o, mode), alone)):
            assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), (rep, i)
        del junk
    del g
    # reuse the arena for fewer, smaller scenes (stale contents must not leak)
    batch.set([scenes[2], scenes[0]])
    out2, offs2, status2 = batch.prepare(tol, mode)
    batch.expand_async(tol, mode, out2.data_ptr(), out2.numel(), offs2.data_ptr(), status2.data_ptr())
    torch.cuda.synchronize()
    o = offs2.cpu().numpy()
    got = _slices(out2, o, mode)
    assert np.array_equal(got[0].view(np.uint8), alone[2].view(np.uint8))
    assert np.array_equal(got[1].view(np.uint8), alone[0].view(np.uint8))
    batch.destroy()


def test_empty_batch(ctx):
    import torch

    from paper_2405_00127_amd import binding as B

    batch = B.Batch(ctx)
    batch.set([])
    offs = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    status = torch.full((2,), 7, dtype=torch.int64, device="cuda")
    batch.expand_async(0.25, S.OUT_LINES, 0, 0, offs.data_ptr(), status.data_ptr())
    torch.cuda.synchronize()
    assert int(offs[0]) == 0 and int(status[0]) == 0 and int(status[1]) == 0
    batch.destroy()


def test_full_size_batch_of_256_scenes(ctx):
    """The 256-scene batch the benchmark times (log-uniform 100..200k
    segments, 8.4 M in total), captured in a graph and replayed: every
    scene's records bit-identical to the scene expanded alone, and sampled
    tags of sampled scenes against the oracle (counts, endpoints, path ids)."""
    import torch

    import oracle as O
    from paper_2405_00127_amd import binding as B

    tol, mode = 0.25, S.OUT_LINES
    _say("full batch: generate")
    scs = S.scene_batch(4, 256, 100, 200_000, mode)
    _say("full batch: segments", sum(s.n_segments() for s in scs))
    stream = torch.cuda.Stream()
    scenes = [ctx.encode(s, stream=stream) for s in scs]
    stream.synchronize()
    alone = [_alone(ctx, s, tol, mode) for s in scenes]
    batch = B.Batch(ctx)
    batch.set(scenes, stream=stream)
    out, offs, status = batch.prepare(tol, mode, stream=stream)
    stream.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        batch.expand_async(tol, mode, out.data_ptr(), out.numel(), offs.data_ptr(), status.data_ptr(),
                           stream=stream)
    for rep in range(2):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        o = offs.cpu().numpy()
        assert int(status[1]) == 0 and int(status[0]) == o[-1] == sum(len(a) for a in alone)
        got = _slices(out, o, mode)
        bad = [i for i in range(len(scs)) if not np.array_equal(got[i].view(np.uint8), alone[i].view(np.uint8))]
        assert not bad, bad
        _say("full batch: replay", rep, "records", int(o[-1]), "all scenes identical to alone")
    # sampled tags of sampled scenes against the oracle
    rng = np.random.default_rng(44)
    worst = 0.0
    import parity as P

    for k in rng.choice(len(scs), 6, replace=False):
        sc = scs[int(k)]
        counts = ctx.counts(scenes[int(k)], tol, mode).cpu().numpy().astype(np.uint32)
        ref = O.expand(sc, emit=False)
        near = P.near_threshold(ref.margins)
        mism = counts != ref.counts
        assert not np.any(mism & ~near)
        go = np.concatenate([[0], np.cumsum(counts.astype(np.int64))])
        for i in np.sort(rng.choice(np.nonzero(~mism)[0], min(50, int((~mism).sum())), replace=False)):
            r = O.expand(sc, emit=True, tag_begin=int(i), tag_end=int(i) + 1, enc=ref.enc)
            gg = got[int(k)][go[i]:go[i + 1]]
            assert len(gg) == len(r.out)
            if len(gg):
                d = max(np.max(np.abs(gg["x0"] - r.out["x0"])), np.max(np.abs(gg["y0"] - r.out["y0"])),
                        np.max(np.abs(gg["x1"] - r.out["x1"])), np.max(np.abs(gg["y1"] - r.out["y1"])))
                worst = max(worst, float(d))
                assert np.all(gg["path"] == r.out["path"])
    _say("full batch: sampled worst endpoint", worst)
    assert worst <= P.ENDPOINT_TOL
    batch.destroy()
