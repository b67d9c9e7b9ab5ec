"""GPU dashing (sx_scene_encode_dashed: the dash passes on the GPU, then the
ordinary expansion) against the oracle's dashing, through the C ABI: the
dashed encoding's tags bit for bit and its points within one FP32 ulp, then
the outlines at the parity bars."""
import sys

import numpy as np
import pytest

import oracle as O
import parity as P
from paper_2405_00127_amd import scenes as S

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2405_00127_amd import binding as B

    torch.cuda.set_device(0)
    c = B.Context(0)
    yield c
    c.close()


def _scene(name):
    if name == "line":
        sc = S.single_path_scene([S.MOVE, S.LINE], [[0, 0], [100, 0]], 2.0, join=S.JOIN_ROUND, cap=S.CAP_BUTT)
        sc.dashes = [(np.array([10, 5], np.float32), -4.0)]
        return sc
    if name == "square":
        sc = S.single_path_scene([S.MOVE, S.LINE, S.LINE, S.LINE, S.CLOSE], [[0, 0], [40, 0], [40, 40], [0, 40]],
                                 1.0, join=S.JOIN_MITER, cap=S.CAP_SQUARE)
        sc.dashes = [(np.array([50, 30], np.float32), 20.0)]
        return sc
    if name == "ulp_corner":
        # a dash boundary 2^-20 before the corner at x = 1010: its part of
        # the first segment has no extent in FP32 and is left out
        sc = S.single_path_scene([S.MOVE, S.LINE, S.LINE], [[1000, 0], [1010, 0], [1010, 10]], 2.0,
                                 join=S.JOIN_MITER, cap=S.CAP_SQUARE)
        sc.dashes = [(np.array([5, 5], np.float32), 2.0 ** -20)]
        return sc
    if name == "ulp_dashes":
        sc = S.single_path_scene([S.MOVE, S.LINE], [[1000, 0], [1010, 0]], 2.0, join=S.JOIN_MITER, cap=S.CAP_ROUND)
        sc.dashes = [(np.array([2.0 ** -20, 1.0], np.float32), 0.0)]
        return sc
    if name == "c1_lines":
        return S.with_dashes(S.scene_c1(1), seed=1)
    if name == "c1_arcs":
        return S.with_dashes(S.scene_c1(1, output_mode=S.OUT_ARCS), seed=1)
    if name == "c1_fills":
        return S.with_dashes(S.with_fills(S.scene_c1(1), 0.5, seed=3), seed=2)
    if name == "map_lines":
        return S.with_dashes(S.scene_c2(2, n_segments=40000, n_paths=400), seed=4, lo=0.5, hi=12.0)
    if name == "stress_arcs":
        return S.with_dashes(S.scene_c3(3, n_cubics=2000), seed=6, lo=2.0, hi=30.0)
    raise KeyError(name)


def _check_encoding(scene, ref):
    tags, data, pm = scene.download()
    assert np.array_equal(tags, ref.tags)
    assert np.array_equal(pm, ref.path_map)
    ulp = np.abs(data.view(np.int32).astype(np.int64) - ref.data.view(np.int32).astype(np.int64))
    assert ulp.max() <= 1 and np.count_nonzero(ulp) <= max(4, 1e-4 * ulp.size), int(np.count_nonzero(ulp))


@pytest.mark.parametrize("name", ["line", "square", "ulp_corner", "ulp_dashes", "c1_lines", "c1_arcs", "c1_fills",
                                  "map_lines", "stress_arcs"])
def test_dashed_scene_parity(ctx, name):
    import torch

    from paper_2405_00127_amd import binding as B

    sc = _scene(name)
    _say("dash parity", name)
    scene = ctx.encode(sc)
    ref_enc = O.encode_dashed(sc)
    _check_encoding(scene, ref_enc)
    assert scene.dash_ms() > 0.0
    mode = sc.output_mode
    recs, n, _ = ctx.expand(scene, sc.tolerance, mode)
    counts = ctx.counts(scene, sc.tolerance, mode).cpu().numpy().astype(np.uint32)
    torch.cuda.synchronize()
    got = B.records_to_numpy(recs, mode)
    assert all(np.all(np.isfinite(got[f])) for f in ("x0", "y0", "x1", "y1"))
    ref = O.expand(sc, enc=ref_enc)
    assert ref.status == 0
    rep = P.compare(counts, got, ref, mode)
    _say(name, rep)
    assert rep.ok(), rep
    assert rep.n_count_mismatch <= max(3, 0.01 * rep.n_tags), rep
    assert P.closed_per_path(got) == 0
    scene.release()


def test_full_size_dashed_map_scene(ctx):
    """The 1M-segment map scene with a dash pattern on every stroke: the
    dashed encoding against the oracle's, then counts of every tag and the
    records of sampled tags."""
    import torch

    from paper_2405_00127_amd import binding as B

    sc = S.with_dashes(S.scene_c2(2), seed=4, lo=0.5, hi=12.0)
    _say("full dashed map: encode")
    scene = ctx.encode(sc)
    _say("full dashed map: dash passes", scene.dash_ms(), "ms,", scene.n_tags, "tags")
    ref_enc = O.encode_dashed(sc)
    _check_encoding(scene, ref_enc)
    recs, n, _ = ctx.expand(scene, sc.tolerance, sc.output_mode)
    counts = ctx.counts(scene).cpu().numpy().astype(np.uint32)
    torch.cuda.synchronize()
    got = B.records_to_numpy(recs, sc.output_mode)
    assert all(np.all(np.isfinite(got[f])) for f in ("x0", "y0", "x1", "y1"))
    ref = O.expand(sc, enc=ref_enc, emit=False)
    near = P.near_threshold(ref.margins)
    mism = counts != ref.counts
    _say("full dashed map: tags", len(counts), "records", n, "mismatch", int(mism.sum()), "near", int(near.sum()))
    assert not np.any(mism & ~near)
    go = np.concatenate([[0], np.cumsum(counts.astype(np.int64))])
    rng = np.random.default_rng(8)
    worst = 0.0
    for i in np.sort(rng.choice(np.nonzero(~mism)[0], 1500, replace=False)):
        r = O.expand(sc, emit=True, tag_begin=int(i), tag_end=int(i) + 1, enc=ref_enc, margins=False)
        g = got[go[i]:go[i + 1]]
        o = r.out
        assert len(o) == len(g)
        if len(g):
            d = max(np.max(np.abs(g["x0"] - o["x0"])), np.max(np.abs(g["y0"] - o["y0"])),
                    np.max(np.abs(g["x1"] - o["x1"])), np.max(np.abs(g["y1"] - o["y1"])))
            worst = max(worst, float(d))
    _say("full dashed map: sampled worst endpoint", worst)
    assert worst <= P.ENDPOINT_TOL
    assert P.closed_per_path(got) == 0
    scene.release()


def test_bad_dash_patterns_are_rejected(ctx):
    from paper_2405_00127_amd import binding as B

    for pat in ([-1.0, 2.0], [float("nan"), 1.0], [2.0 ** -12, 2.0 ** -12]):
        sc = _scene("line")
        sc.dashes = [(np.array(pat, np.float32), 0.0)]
        with pytest.raises(B.StrokexError) as ei:
            ctx.encode(sc)
        assert ei.value.code == B.SX_EINVAL
    # coordinates beyond 2^24 units, and a segment that would need more than
    # 2^20 chunks of dashes (a pattern of 2^-10 units along 1.6e7 units)
    for pts, pat in (([[0, 0], [3.0e7, 0]], [1.0, 1.0]), ([[0, 0], [1.6e7, 0]], [2.0 ** -11, 2.0 ** -11])):
        sc = S.single_path_scene([S.MOVE, S.LINE], pts, 1.0, join=S.JOIN_ROUND, cap=S.CAP_BUTT)
        sc.dashes = [(np.array(pat, np.float32), 0.0)]
        with pytest.raises(B.StrokexError) as ei:
            ctx.encode(sc)
        assert ei.value.code == B.SX_EINVAL
    sc = _scene("line")
    sc.dashes = [(np.array([0.0, 0.0], np.float32), 0.0)]  # total length 0: solid
    scene = ctx.encode(sc)
    recs, n, _ = ctx.expand(scene)
    assert n == 4
