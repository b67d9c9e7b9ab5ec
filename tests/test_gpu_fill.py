"""Fill flattening on the GPU (HIP, gfx950) against the FP64 oracle, through
the C ABI: the same bars as the strokes (encoding bit-exact, counts identical
except at oracle decisions within the margin thresholds, endpoints within
1e-3 px, path ids equal, outlines closed per path), for fills alone, fills
mixed with strokes, fills under a non-similarity transform, and the
1M-segment map scene drawn as fills in the benchmark's launch configuration."""
import sys

import numpy as np
import pytest

import oracle as O
import parity as P
from paper_2405_00127_amd import scenes as S

pytestmark = pytest.mark.gpu

SHEAR = [1.0, 0.2, 0.5, 0.9, 10.0, -5.0]


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


def _expand(ctx, sc, mode=None):
    import torch

    from paper_2405_00127_amd import binding as B

    mode = sc.output_mode if mode is None else mode
    scene = ctx.encode(sc)
    recs, n, _ = ctx.expand(scene, sc.tolerance, mode)
    counts = ctx.counts(scene, sc.tolerance, mode).cpu().numpy().astype(np.uint32)
    torch.cuda.synchronize()
    return scene, counts, B.records_to_numpy(recs, mode)


def _scene(name):
    if name == "c1_fill_lines":
        return S.with_fills(S.scene_c1(1))
    if name == "c1_fill_arcs":
        return S.with_fills(S.scene_c1(1, output_mode=S.OUT_ARCS))
    if name == "c1_mixed_shear":
        return S.with_fills(S.scene_c1(1), 0.5, seed=3, xform=SHEAR)
    if name == "c2_mixed":
        return S.with_fills(S.scene_c2(2, n_segments=40000, n_paths=400), 0.5, seed=5)
    if name == "c3_fill_lines":
        return S.with_fills(S.scene_c3(3, n_cubics=3000, output_mode=S.OUT_LINES))
    if name == "c3_fill_arcs":
        return S.with_fills(S.scene_c3(3, n_cubics=3000))
    raise KeyError(name)


NAMES = ["c1_fill_lines", "c1_fill_arcs", "c1_mixed_shear", "c2_mixed", "c3_fill_lines", "c3_fill_arcs"]


@pytest.mark.parametrize("name", ["c1_mixed_shear", "c2_mixed"])
def test_fill_encoding_bit_exact(ctx, name):
    sc = _scene(name)
    _say("fill encoding", name)
    scene = ctx.encode(sc)
    tags, data, pm = scene.download()
    e = O.encode(sc)
    assert np.array_equal(tags, e.tags)
    assert np.array_equal(data.view(np.uint32), e.data.view(np.uint32))
    assert np.array_equal(pm, e.path_map)


@pytest.mark.parametrize("name", NAMES)
def test_fill_outline_parity(ctx, name):
    sc = _scene(name)
    _say("fill parity", name, "segments", sc.n_segments())
    scene, counts, recs = _expand(ctx, sc)
    ref = O.expand(sc)
    assert ref.status == 0
    rep = P.compare(counts, recs, ref, sc.output_mode)
    _say(name, rep)
    assert rep.n_unexplained == 0, rep
    assert rep.worst_endpoint <= P.ENDPOINT_TOL, rep
    assert rep.worst_sweep <= P.SWEEP_TOL, rep
    assert rep.bad_path_ids == 0
    assert rep.n_count_mismatch <= max(3, 0.01 * rep.n_tags), rep
    assert P.closed_per_path(recs) == 0


def test_full_size_map_scene_as_fills(ctx):
    """The 1M-segment map scene with every path filled, in the launch
    configuration the benchmark times: counts of every tag against the
    oracle's count pass, records of sampled tags against the oracle run tag
    by tag, every outline closed."""
    sc = S.with_fills(S.scene_c2(2))
    _say("full fill: encode")
    scene, counts, recs = _expand(ctx, sc)
    _say("full fill: oracle counts")
    ref = O.expand(sc, emit=False)
    near = P.near_threshold(ref.margins)
    mism = counts != ref.counts
    _say("full fill: tags", len(counts), "mismatch", int(mism.sum()), "near", int(near.sum()))
    assert not np.any(mism & ~near)
    assert mism.sum() <= 1e-3 * len(counts)
    go = np.concatenate([[0], np.cumsum(counts.astype(np.int64))])
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(np.nonzero(~mism)[0], 3000, replace=False))
    worst = 0.0
    for i in sample:
        r = O.expand(sc, emit=True, tag_begin=int(i), tag_end=int(i) + 1, enc=ref.enc)
        g = recs[go[i] : go[i + 1]]
        o = r.out
        assert len(o) == len(g)
        if len(g):
            d = max(np.max(np.abs(g["x0"] - o["x0"])), np.max(np.abs(g["y0"] - o["y0"])),
                    np.max(np.abs(g["x1"] - o["x1"])), np.max(np.abs(g["y1"] - o["y1"])))
            worst = max(worst, float(d))
            assert np.all(g["path"] == o["path"])
    _say("full fill: sampled worst endpoint", worst)
    assert worst <= P.ENDPOINT_TOL
    assert P.closed_per_path(recs) == 0


@pytest.mark.parametrize("case", ["fill_shear_ok", "stroke_shear", "fill_singular", "reserved_flag"])
def test_fill_validation(ctx, case):
    from paper_2405_00127_amd import binding as B

    st = S.make_styles([1.0], 2, 0)
    xf = S.identity_xforms()
    if case in ("fill_shear_ok", "fill_singular"):
        st["flags"] = S.STYLE_FILL
    if case in ("fill_shear_ok", "stroke_shear"):
        xf = np.array([SHEAR], np.float32)
    if case == "fill_singular":
        xf = np.array([[1, 2, 2, 4, 0, 0]], np.float32)
    if case == "reserved_flag":
        st["flags"] = 2
    b = S.SceneBuilder()
    b.add_path([0, 1, 1], [[0, 0], [10, 0], [10, 10]], 0, 0)
    sc = b.build(st, xf)
    if case == "fill_shear_ok":
        scene, counts, recs = _expand(ctx, sc)
        ref = O.expand(sc)
        assert ref.status == 0
        assert np.array_equal(counts, ref.counts)
        assert len(recs) == 3 and P.closed_per_path(recs) == 0
        return
    with pytest.raises(B.StrokexError) as ei:
        ctx.encode(sc)
    assert ei.value.code == B.SX_EINVAL
