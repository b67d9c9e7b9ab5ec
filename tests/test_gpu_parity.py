"""GPU (HIP, gfx950) vs FP64 oracle parity, through the C ABI.

Bars: encoding and monoids bit-exact; output offsets bit-exact where the
counts agree; counts identical except at oracle decisions within the margin
thresholds of ``parity`` (1e-9: both sides decide in FP64); endpoints within
1e-3 px; arcs' bulge within 1e-3 px; path ids equal; outlines closed
bit-exactly per path."""
import math
import sys

import numpy as np
import pytest

import oracle as O
import parity as P
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


def _expand(ctx, sc, mode=None):
    import torch

    from paper_2405_00127_amd import binding as B

    mode = sc.output_mode if mode is None else mode
    scene = ctx.encode(sc)
    recs, n, _ = ctx.expand(scene, sc.tolerance, mode)
    counts = ctx.counts(scene, sc.tolerance, mode).cpu().numpy().astype(np.uint32)
    torch.cuda.synchronize()
    return scene, counts, B.records_to_numpy(recs, mode)


# ------------------------------------------------------------- encoding
@pytest.mark.parametrize("name", ["c1", "c2small", "c3small"])
def test_encoding_bit_exact(ctx, name):
    sc = {"c1": lambda: S.scene_c1(1), "c2small": lambda: S.scene_c2(2, n_segments=30000, n_paths=300),
          "c3small": lambda: S.scene_c3(3, n_cubics=500)}[name]()
    _say("encoding", name)
    scene = ctx.encode(sc)
    tags, data, pm = scene.download()
    e = O.encode(sc)
    assert np.array_equal(tags, e.tags)
    assert np.array_equal(data.view(np.uint32), e.data.view(np.uint32))
    assert np.array_equal(pm, e.path_map)


# --------------------------------------------------------------- scans
@pytest.mark.parametrize("n", [1, 2, 15, 16, 17, 4095, 4096, 4097, 65536 * 4 + 3, 1 << 20])
def test_scan_u32_bit_exact(ctx, n):
    import torch

    _say("scan_u32 n =", n)
    rng = np.random.default_rng(n)
    v = rng.integers(0, 5000, n).astype(np.uint32)
    t = torch.from_numpy(v.view(np.int32)).cuda()
    out = ctx.scan_u32(t).cpu().numpy().astype(np.uint64)
    ref = np.concatenate([[0], np.cumsum(v.astype(np.uint64))])
    assert np.array_equal(out, ref)


def test_scan_u32_repeated_launches(ctx):
    import torch

    v = np.arange(50000, dtype=np.uint32) % 7
    t = torch.from_numpy(v.view(np.int32)).cuda()
    ref = np.concatenate([[0], np.cumsum(v.astype(np.uint64))])
    for _ in range(5):
        assert np.array_equal(ctx.scan_u32(t).cpu().numpy().astype(np.uint64), ref)


@pytest.mark.parametrize("name", ["c1", "c2", "tiny", "tile_edges"])
def test_monoids_bit_exact(ctx, name):
    if name == "c1":
        sc = S.scene_c1(1)
    elif name == "c2":
        sc = S.scene_c2(2)
    elif name == "tiny":
        sc = S.single_path_scene([0, 1], [[0, 0], [1, 0]], 1.0)
    else:
        # 4096-tag tiles: paths sized so tag counts straddle tile boundaries
        b = S.SceneBuilder()
        rng = np.random.default_rng(0)
        for k, n in enumerate([4094, 1, 4096, 4095, 2, 8191]):
            pts = np.cumsum(rng.uniform(-3, 3, (n + 1, 2)), 0) + 500
            b.add_path([0] + [1] * n, pts, k % 3, 0)
        sc = b.build(S.make_styles([1.0, 2.0, 3.0], S.JOIN_ROUND, S.CAP_BUTT))
    _say("monoids", name)
    scene = ctx.encode(sc)
    e = O.encode(sc)
    for rep in range(3):  # repeated launches reuse the look-back state
        m = ctx.monoids(scene).cpu().numpy().view(np.uint32)
        assert np.array_equal(m, O.monoids(e.tags)), rep


# ------------------------------------------------------------- outlines
def _scene(name):
    if name == "c1_lines":
        return S.scene_c1(1)
    if name == "c1_arcs":
        return S.scene_c1(1, output_mode=S.OUT_ARCS)
    if name == "c2_lines":
        return S.scene_c2(2, n_segments=40000, n_paths=400)
    if name == "c2_arcs":
        return S.scene_c2(2, n_segments=40000, n_paths=400, output_mode=S.OUT_ARCS)
    if name == "c3_arcs":
        return S.scene_c3(3, n_cubics=3000)
    if name == "c3_lines":
        return S.scene_c3(3, n_cubics=3000, output_mode=S.OUT_LINES)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["c1_lines", "c1_arcs", "c2_lines", "c2_arcs", "c3_arcs", "c3_lines"])
def test_outline_parity(ctx, name):
    sc = _scene(name)
    _say("parity", name, "segments", sc.n_segments())
    scene, counts, recs = _expand(ctx, sc)
    ref = O.expand(sc)
    assert ref.status == 0
    rep = P.compare(counts, recs, ref, sc.output_mode)
    _say(name, rep)
    assert rep.n_unexplained == 0, rep
    assert rep.worst_endpoint <= P.ENDPOINT_TOL, rep
    assert rep.worst_sweep <= P.SWEEP_TOL, rep
    assert rep.bad_path_ids == 0
    # near-threshold exclusions stay rare
    assert rep.n_count_mismatch <= max(3, 0.01 * rep.n_tags), rep
    assert P.closed_per_path(recs) == 0


def _tile_edge_scene(name, mode):
    """Scenes whose piece counts fall on and around the 256-piece tiles of the
    piece launch (lines are one piece each; open subpaths end in a cap marker,
    a tag without pieces whose tail joins the tile of the piece before it)."""
    rng = np.random.default_rng({"exact256": 1, "exact512": 2, "mixed": 3}[name])
    b = S.SceneBuilder()

    def poly(n, closed=False):
        pts = np.cumsum(rng.uniform(-4, 4, (n + 1, 2)), 0) + 300
        b.add_path([S.MOVE] + [S.LINE] * n + ([S.CLOSE] if closed else []), pts, int(rng.integers(0, 3)))

    if name == "exact256":
        poly(256)
    elif name == "exact512":
        poly(200)
        poly(312)
    else:
        for n in [255, 1, 256, 257, 511, 1, 512]:
            poly(n, closed=bool(rng.integers(0, 2)))
        for _ in range(600):  # one piece and one marker each
            poly(1)
        for _ in range(40):  # wide cubics: several pieces per tag, straddling tiles
            p = rng.uniform(0, 200, (4, 2))
            b.add_path([S.MOVE, S.CUBIC], p, 2)
        poly(300)
    styles = S.make_styles([0.5, 2.0, 12.0], S.JOIN_ROUND, S.CAP_ROUND)
    return b.build(styles, name=name, output_mode=mode)


@pytest.mark.parametrize("mode", [S.OUT_LINES, S.OUT_ARCS])
@pytest.mark.parametrize("name", ["exact256", "exact512", "mixed"])
def test_piece_tile_edges(ctx, name, mode):
    """A tile of the piece launch holds 256 pieces and owns the slots from its
    first piece to the next tile's first (with the tails between them):
    scenes of exactly one and two full tiles, and polylines of 255, 256,
    257, 511 and 512 lines, single-line subpaths and multi-piece cubics whose
    pieces straddle tile boundaries, against the oracle."""
    sc = _tile_edge_scene(name, mode)
    scene, counts, recs = _expand(ctx, sc)
    ref = O.expand(sc)
    assert ref.status == 0
    n_pieces = len(ref.pieces)
    _say("tile edges", name, mode, "tags", len(counts), "pieces", n_pieces)
    assert n_pieces == {"exact256": 256, "exact512": 512}.get(name, n_pieces)
    rep = P.compare(counts, recs, ref, sc.output_mode)
    assert rep.n_unexplained == 0, rep
    assert rep.worst_endpoint <= P.ENDPOINT_TOL, rep
    assert rep.worst_sweep <= P.SWEEP_TOL, rep
    assert rep.bad_path_ids == 0
    assert P.closed_per_path(recs) == 0


def test_offsets_are_the_scan_of_the_counts(ctx):
    sc = _scene("c2_lines")
    scene = ctx.encode(sc)
    c = ctx.counts(scene).cpu().numpy().astype(np.uint64)
    o = ctx.offsets(scene).cpu().numpy().astype(np.uint64)
    assert np.array_equal(o, np.concatenate([[0], np.cumsum(c)]))


@pytest.mark.parametrize("mode", [S.OUT_LINES, S.OUT_ARCS])
def test_full_size_c2_counts_and_samples(ctx, mode):
    """The 1M-segment map scene, lines and arcs, at the default launch
    parameters (test_gpu_tuning shows every launch configuration the tuner
    can pick gives these records bit for bit): counts of every tag against
    the oracle (count-only pass) and the records of sampled tags against the
    oracle run tag by tag (endpoints, arc bulge, path ids)."""
    sc = S.scene_c2(2, output_mode=mode)
    _say("full c2: encode", mode)
    scene, counts, recs = _expand(ctx, sc)
    _say("full c2: oracle counts")
    ref = O.expand(sc, emit=False)
    near = P.near_threshold(ref.margins)
    mism = counts != ref.counts
    _say("full c2: tags", len(counts), "mismatch", int(mism.sum()), "near", int(near.sum()))
    assert not np.any(mism & ~near)
    assert mism.sum() <= 1e-3 * len(counts)
    go = np.concatenate([[0], np.cumsum(counts.astype(np.int64))])
    rng = np.random.default_rng(9)
    sample = np.sort(rng.choice(np.nonzero(~mism)[0], 3000, replace=False))
    worst = worst_b = 0.0
    enc = ref.enc
    for i in sample:
        r = O.expand(sc, emit=True, tag_begin=int(i), tag_end=int(i) + 1, enc=enc)
        g = recs[go[i] : go[i + 1]]
        o = r.out
        assert len(o) == len(g)
        if len(g):
            d = max(np.max(np.abs(g["x0"] - o["x0"])), np.max(np.abs(g["y0"] - o["y0"])),
                    np.max(np.abs(g["x1"] - o["x1"])), np.max(np.abs(g["y1"] - o["y1"])))
            worst = max(worst, float(d))
            if mode == S.OUT_ARCS:
                worst_b = max(worst_b, float(np.max(np.abs(P.arc_bulge(g) - P.arc_bulge(o)))))
            assert np.all(g["path"] == o["path"])
    _say("full c2: sampled worst endpoint", worst, "bulge", worst_b)
    assert worst <= P.ENDPOINT_TOL
    assert worst_b <= P.SWEEP_TOL
    assert P.closed_per_path(recs) == 0


def test_full_size_c3_counts_and_samples(ctx):
    """The 100,000-cubic stress scene (cusps, near-cusps, loops, degenerate
    control points; half-widths 5-50 px; tolerance 0.1 px; arcs) in one
    launch: counts of every tag against the oracle, the records of sampled
    windows of tags against the oracle run on those tags (endpoints, arc
    bulge, path ids), the outlines closed per path, and the offset records of
    sampled tags within tolerance of the exact FP64 parallel curves."""
    import exact_stroke as X

    _say("full c3: generate")
    sc = S.scene_c3(3)
    _say("full c3: expand", sc.n_segments(), "segments")
    scene, counts, recs = _expand(ctx, sc)
    _say("full c3: oracle counts")
    ref = O.expand(sc, emit=False)
    near = P.near_threshold(ref.margins)
    mism = counts != ref.counts
    _say("full c3: tags", len(counts), "records", int(counts.sum()), "mismatch", int(mism.sum()), "near",
         int(near.sum()))
    assert not np.any(mism & ~near)
    assert mism.sum() <= 1e-3 * len(counts)
    go = np.concatenate([[0], np.cumsum(counts.astype(np.int64))])
    rng = np.random.default_rng(33)
    enc = ref.enc
    mon = O.monoids(enc.tags)
    worst = worst_b = worst_x = 0.0
    for a in np.sort(rng.choice(len(counts) - 40, 40, replace=False)):
        a = int(a)
        r = O.expand(sc, emit=True, tag_begin=a, tag_end=a + 40, enc=enc)
        ro = np.concatenate([[0], np.cumsum(r.counts[a:a + 40].astype(np.int64))])
        for i in range(a, a + 40):
            if mism[i] or near[i]:
                continue
            g = recs[go[i]:go[i + 1]]
            o = r.out[ro[i - a]:ro[i - a + 1]]
            assert len(o) == len(g)
            if not len(g):
                continue
            d = max(np.max(np.abs(g["x0"] - o["x0"])), np.max(np.abs(g["y0"] - o["y0"])),
                    np.max(np.abs(g["x1"] - o["x1"])), np.max(np.abs(g["y1"] - o["y1"])))
            worst = max(worst, float(d))
            worst_b = max(worst_b, float(np.max(np.abs(P.arc_bulge(g) - P.arc_bulge(o)))))
            assert np.all(g["path"] == o["path"])
            if (enc.tags[i] & 4) == 0 and i % 8 == 0:
                # offsets of this segment against the exact parallel curves
                off = g[o["kind"] == O.KIND_OFFSET]
                xf = sc.xforms[enc.xform_stream[mon[3][i]]]
                w = float(sc.styles[enc.style_stream[mon[2][i]]]["half_width"])
                P_, W = X.world_segment(enc.data, mon[0][i], enc.tags[i], xf)
                A, B_, cusps = X.dense_offsets(P_, w, 0.02)
                refpts = np.concatenate([A, B_] + [X.circle_pts(c, w) for c in cusps])
                pts, _ = X.sample_outputs(off["x0"].astype(np.float64), off["y0"].astype(np.float64),
                                          off["x1"].astype(np.float64), off["y1"].astype(np.float64),
                                          off["curv"].astype(np.float64), 0.05)
                worst_x = max(worst_x, X.max_dist(pts, refpts)[0])
    _say("full c3: sampled worst endpoint", worst, "bulge", worst_b, "distance to exact", worst_x)
    assert worst <= P.ENDPOINT_TOL
    assert worst_b <= P.SWEEP_TOL
    assert worst_x <= sc.tolerance
    assert P.closed_per_path(recs) == 0


@pytest.mark.parametrize("name", ["c1_lines", "c3_arcs"])
def test_gpu_offsets_within_tolerance_of_exact_curve(ctx, name):
    """Every GPU offset record within tau of the FP64 exact parallel curves
    (independent dense sampling), on a subset of segments."""
    import exact_stroke as X

    sc = _scene(name)
    if name == "c1_lines":
        sc = sc.subset(range(3))
    else:
        sc = S.scene_c3(3, n_cubics=200)
    scene, counts, recs = _expand(ctx, sc)
    ref = O.expand(sc)
    go = np.concatenate([[0], np.cumsum(counts.astype(np.int64))])
    oo = ref.offsets().astype(np.int64)
    mon = O.monoids(ref.enc.tags)
    worst = 0.0
    for i in np.nonzero(((ref.enc.tags & 4) == 0) & (counts == ref.counts))[0]:
        kinds = ref.out[oo[i] : oo[i + 1]]["kind"]
        g = recs[go[i] : go[i + 1]][kinds == O.KIND_OFFSET]
        xf = sc.xforms[ref.enc.xform_stream[mon[3][i]]]
        w = float(sc.styles[ref.enc.style_stream[mon[2][i]]]["half_width"])
        P_, W = X.world_segment(ref.enc.data, mon[0][i], ref.enc.tags[i], xf)
        A, B_, cusps = X.dense_offsets(P_, w, 0.02)
        refpts = np.concatenate([A, B_] + [X.circle_pts(c, w) for c in cusps])
        pts, _ = X.sample_outputs(g["x0"].astype(np.float64), g["y0"].astype(np.float64),
                                  g["x1"].astype(np.float64), g["y1"].astype(np.float64),
                                  g["curv"].astype(np.float64) if sc.output_mode == S.OUT_ARCS else None, 0.05)
        worst = max(worst, X.max_dist(pts, refpts)[0])
    _say(name, "worst distance to exact", worst)
    assert worst <= sc.tolerance


# ------------------------------------------------------ edge behaviour
def test_too_small_buffer_reports_the_count(ctx):
    import torch

    from paper_2405_00127_amd import binding as B

    sc = S.scene_c1(1).subset(range(3))
    scene = ctx.encode(sc)
    buf = torch.zeros(100, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.StrokexError) as ei:
        ctx.expand_into(scene, buf.data_ptr(), buf.numel(), sc.tolerance, S.OUT_LINES)
    assert ei.value.code == B.SX_ETOOSMALL
    assert ei.value.required > 5
    assert int(buf.sum()) == 0  # nothing written
    recs, n, _ = ctx.expand(scene)
    assert n == ei.value.required


def test_async_workspace_overflow_is_reported_then_resized(ctx):
    """A scene needing more slots and emission items than its initial
    workspace: the asynchronous call reports it and emits nothing; one
    synchronous call resizes the workspace; the asynchronous call then
    matches it bit for bit."""
    import torch

    from paper_2405_00127_amd import binding as B

    sc = S.scene_c3(3, n_cubics=500)
    mode = sc.output_mode
    _say("async overflow", sc.name)
    scene = ctx.encode(sc)
    rec = B.RECORD_BYTES[mode]
    buf = torch.zeros(4_000_000 * rec, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(2, dtype=torch.int64, device="cuda")
    ctx.expand_async(scene, buf.data_ptr(), buf.numel(), cnt.data_ptr(), sc.tolerance, mode)
    torch.cuda.synchronize()
    need = int(cnt[1])
    assert need != 0
    recs, n, _ = ctx.expand(scene, sc.tolerance, mode)
    assert int(buf[: n * rec].count_nonzero()) == 0  # nothing was emitted
    ref = B.records_to_numpy(recs, mode).copy()
    buf.zero_()
    cnt.zero_()
    ctx.expand_async(scene, buf.data_ptr(), buf.numel(), cnt.data_ptr(), sc.tolerance, mode)
    torch.cuda.synchronize()
    assert int(cnt[0]) == n and int(cnt[1]) == 0
    got = B.records_to_numpy(buf[: n * rec].view(torch.float32).view(-1, rec // 4), mode)
    assert np.array_equal(got.view(np.uint8), ref.view(np.uint8))


def test_repeated_runs_are_bit_identical(ctx):
    sc = _scene("c1_arcs")
    _, c1, r1 = _expand(ctx, sc)
    _, c2, r2 = _expand(ctx, sc)
    assert np.array_equal(c1, c2)
    assert np.array_equal(r1.view(np.uint8), r2.view(np.uint8))


def test_empty_scene(ctx):
    sc = S.SceneBuilder().build(S.make_styles([1.0], S.JOIN_ROUND, S.CAP_BUTT))
    scene = ctx.encode(sc)
    recs, n, _ = ctx.expand(scene, 0.25, S.OUT_LINES)
    assert n == 0


@pytest.mark.parametrize("bad", ["no_move", "nan", "neg_width", "shear", "bad_style_ix"])
def test_invalid_inputs_are_rejected(ctx, bad):
    from paper_2405_00127_amd import binding as B

    verbs, pts, st, xf, six = [0, 1], [[0, 0], [1, 0]], S.make_styles([1.0], 2, 0), S.identity_xforms(), 0
    if bad == "no_move":
        verbs, pts = [1], [[1, 0]]
    elif bad == "nan":
        pts = [[0, 0], [math.nan, 0]]
    elif bad == "neg_width":
        st = S.make_styles([-1.0], 2, 0)
    elif bad == "shear":
        xf = np.array([[1, 0, 0.5, 1, 0, 0]], np.float32)
    else:
        six = 3
    b = S.SceneBuilder()
    b.add_path(verbs, pts, six, 0)
    sc = b.build(st, xf)
    with pytest.raises(B.StrokexError) as ei:
        ctx.encode(sc)
    assert ei.value.code == B.SX_EINVAL
    bad_tol = S.single_path_scene([0, 1], [[0, 0], [1, 0]], 1.0)
    scene = ctx.encode(bad_tol)
    with pytest.raises(B.StrokexError):
        ctx.expand(scene, tolerance=0.0)


@pytest.mark.parametrize("name,factor", [("c1", 1.5), ("c2", 1.1)])
def test_host_estimate_of_records(ctx, name, factor):
    """sx_scene_estimate (host only: Wang's formula per curve, inflated per
    stroke side, plus join / cap bounds) covers these scenes' exact need with
    room to spare; on cusp-heavy scenes it is a heuristic and may fall short."""
    sc = {"c1": lambda: S.scene_c1(1), "c2": lambda: S.scene_c2(2, n_segments=40000, n_paths=400)}[name]()
    scene = ctx.encode(sc)
    need = int(O.expand(sc, emit=False).counts.sum())
    est = ctx.estimate(scene, sc.tolerance, sc.output_mode)
    _say("estimate", name, est, "need", need)
    assert est >= factor * need
    assert est == ctx.estimate(scene, sc.tolerance, sc.output_mode)  # deterministic
    assert ctx.estimate(scene, 2 * sc.tolerance, sc.output_mode) < est  # coarser tolerance, fewer records
