"""End-to-end pins of the oracle's outlines against the exact FP64 geometry
(independent dense sampling in ``exact_stroke``), hand-derived cases and
invariants.  CPU only."""
import collections
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial import cKDTree

import exact_stroke as X
import oracle as O
from paper_2405_00127_amd import scenes as S

HAND = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_derived.json")))


def _lines(res):
    o = res.out
    return np.stack([o["x0"], o["y0"], o["x1"], o["y1"]], 1)


@pytest.mark.parametrize("case,join,cap", [("line_butt", S.JOIN_ROUND, S.CAP_BUTT),
                                           ("line_square", S.JOIN_ROUND, S.CAP_SQUARE),
                                           ("right_angle_bevel", S.JOIN_BEVEL, S.CAP_BUTT),
                                           ("right_angle_miter", S.JOIN_MITER, S.CAP_BUTT)])
def test_hand_derived_outlines(case, join, cap):
    c = HAND[case]
    sc = S.single_path_scene(c["verbs"], c["pts"], c["half_width"], join=join, cap=cap)
    r = O.expand(sc)
    assert r.status == 0
    got = _lines(r)
    want = np.array(c["lines"], dtype=np.float64)
    assert got.shape == want.shape
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("ang", [0.0, 0.3, 2.0, -2.7])
def test_offset_of_a_line_is_a_line(ang):
    d = np.array([math.cos(ang), math.sin(ang)])
    p0 = np.array([50.0, 60.0])
    p1 = p0 + 137.25 * d
    for verbs, pts in [([0, 1], [p0, p1]), ([0, 3], [p0, p0 + 0.2 * (p1 - p0), p0 + 0.7 * (p1 - p0), p1])]:
        sc = S.single_path_scene(verbs, pts, 7.5, cap=S.CAP_BUTT)
        r = O.expand(sc)
        off = r.out[r.out["kind"] == O.KIND_OFFSET]
        assert len(off) == 2
        p0f = np.asarray(sc.pts[0], np.float64)
        p1f = np.asarray(sc.pts[-1], np.float64)
        t = p1f - p0f
        t /= np.linalg.norm(t)
        N = np.array([t[1], -t[0]])
        a = off[0]
        b = off[1]
        assert np.allclose([a["x0"], a["y0"]], p0f + 7.5 * N, atol=1e-9)
        assert np.allclose([a["x1"], a["y1"]], p1f + 7.5 * N, atol=1e-9)
        assert np.allclose([b["x0"], b["y0"]], p1f - 7.5 * N, atol=1e-9)
        assert np.allclose([b["x1"], b["y1"]], p0f - 7.5 * N, atol=1e-9)


def _arc_cubic(R, alpha, c=(0.0, 0.0)):
    k = 4 / 3 * math.tan(alpha / 4) * R
    p0 = np.array([R, 0.0])
    p3 = R * np.array([math.cos(alpha), math.sin(alpha)])
    p1 = p0 + k * np.array([0.0, 1.0])
    p2 = p3 + k * np.array([math.sin(alpha), -math.cos(alpha)])
    return np.array([p0, p1, p2, p3]) + np.asarray(c)


@pytest.mark.parametrize("mode", [S.OUT_LINES, S.OUT_ARCS])
def test_offset_of_an_arc_is_a_concentric_arc(mode):
    R, alpha, w, tol = 100.0, 0.3, 10.0, 0.25
    P = _arc_cubic(R, alpha)
    sc = S.single_path_scene([0, 3], P, w, cap=S.CAP_BUTT, tolerance=tol, output_mode=mode)
    r = O.expand(sc)
    off = r.out[r.out["kind"] == O.KIND_OFFSET]
    rad = np.hypot(np.r_[off["x0"], off["x1"]], np.r_[off["y0"], off["y1"]])
    # CCW arc: side A (right normal) is the outside, side B the inside
    assert np.all(np.abs(np.sort(rad)[len(rad) // 2:] - (R + w)) < 1e-4)
    assert np.all(np.abs(np.sort(rad)[: len(rad) // 2] - (R - w)) < 1e-4)
    if mode == S.OUT_LINES:
        # Section 2.1 metric with the parallel-curve density sqrt(|k| |1 + h k|)
        tf = 0.65 * tol
        L = R * alpha
        for h in (+w, -w):
            kappa = 1.0 / R
            n = math.ceil(L * math.sqrt(kappa * abs(1 + h * kappa)) * math.sqrt(1 / (8 * tf)))
            r_side = R + h
            cnt = np.sum(np.abs(np.hypot(off["x0"], off["y0"]) - r_side) < 1e-3)
            assert cnt == n
    else:
        assert np.all(np.abs(np.abs(off["curv"]) - 1.0 / np.where(
            np.abs(np.hypot(off["x0"], off["y0"]) - (R + w)) < 1e-3, R + w, R - w)) < 1e-6)


def test_zero_width_stroke_uses_the_plain_density():
    # h = 0: Section 2.2 density sqrt|kappa|; for an arc n = s sqrt(kappa / 8 d)
    R, alpha, tol = 200.0, 0.4, 0.25
    sc = S.single_path_scene([0, 3], _arc_cubic(R, alpha), 0.0, cap=S.CAP_BUTT, tolerance=tol)
    r = O.expand(sc)
    off = r.out[r.out["kind"] == O.KIND_OFFSET]
    n = math.ceil(R * alpha * math.sqrt((1 / R) / (8 * 0.65 * tol)))
    assert len(off) == 2 * n


def _closed_per_path(res, exact=True):
    starts = collections.defaultdict(collections.Counter)
    ends = collections.defaultdict(collections.Counter)
    for o in res.out:
        starts[int(o["path"])][(o["x0"], o["y0"])] += 1
        ends[int(o["path"])][(o["x1"], o["y1"])] += 1
    for p in starts:
        assert starts[p] == ends[p], p


@pytest.mark.parametrize("name", ["c1", "c2", "c3lines", "c3arcs"])
def test_outlines_are_closed(name):
    sc = _small_scene(name)
    r = O.expand(sc)
    assert r.status == 0
    assert len(r.out) == int(r.counts.sum())
    _closed_per_path(r)


def _small_scene(name):
    if name == "c1":
        return S.scene_c1(1).subset(range(4))
    if name == "c2":
        return S.scene_c2(2, n_segments=4000, n_paths=40)
    if name == "c3lines":
        return S.scene_c3(3, n_cubics=60, per_path=10, output_mode=S.OUT_LINES)
    if name == "c3arcs":
        return S.scene_c3(3, n_cubics=60, per_path=10, output_mode=S.OUT_ARCS)
    raise KeyError(name)


def test_counts_without_emission_match():
    sc = _small_scene("c3arcs")
    a = O.expand(sc, emit=True)
    b = O.expand(sc, emit=False)
    assert np.array_equal(a.counts, b.counts)
    assert len(b.out) == 0


def test_pieces_are_a_dyadic_cover():
    sc = _small_scene("c1")
    r = O.expand(sc)
    for tag in np.unique(r.pieces["tag"]):
        p = r.pieces[r.pieces["tag"] == tag]
        assert p["t0"][0] == 0.0 and p["t1"][-1] == 1.0
        assert np.all(p["t0"][1:] == p["t1"][:-1])
        dt = p["t1"] - p["t0"]
        e = np.log2(dt)
        assert np.all(e == np.round(e))  # powers of two (two-word stack)
        assert np.all(np.mod(p["t0"] / dt, 1.0) == 0.0)
        assert np.all(dt >= 2.0**-16)


def _segment_geometry(sc, res):
    enc = res.enc
    mon = O.monoids(enc.tags)
    xfs = sc.xforms[enc.xform_stream]
    sty = sc.styles[enc.style_stream]
    for i in np.nonzero((enc.tags & X.TAG_END) == 0)[0]:
        xf = xfs[mon[3][i]]
        w = float(sty[mon[2][i]]["half_width"]) * math.sqrt(abs(float(xf[0]) * float(xf[3]) - float(xf[1]) * float(xf[2])))
        P, W = X.world_segment(enc.data, mon[0][i], enc.tags[i], xf)
        yield i, P, W, w


@pytest.mark.parametrize("name", ["c1", "c2", "c3lines", "c3arcs"])
def test_offsets_within_tolerance_of_exact_parallel_curves(name):
    """O13.2: every offset output within tau of the exact parallel curves of its
    own segment, and every exact parallel-curve point within tau of the
    segment's offset outputs (both directions of the Hausdorff distance)."""
    sc = _small_scene(name)
    r = O.expand(sc)
    offs = r.offsets()
    tol = sc.tolerance
    worst_fwd = worst_back = 0.0
    for i, P, W, w in _segment_geometry(sc, r):
        o = r.out[offs[i] : offs[i + 1]]
        o = o[o["kind"] == O.KIND_OFFSET]
        A, B, cusps = X.dense_offsets(P, w, 0.02)
        ref = np.concatenate([A, B] + [X.circle_pts(c, w) for c in cusps])
        pts, _ = X.sample_outputs(o["x0"], o["y0"], o["x1"], o["y1"],
                                  o["curv"] if sc.output_mode == S.OUT_ARCS else None, 0.05)
        d, _ = X.max_dist(pts, ref)
        worst_fwd = max(worst_fwd, d)
        if not cusps:
            db, _ = X.max_dist(np.concatenate([A, B]), pts)
            worst_back = max(worst_back, db)
    assert worst_fwd <= tol, worst_fwd
    assert worst_back <= tol + 0.05, worst_back  # + output sampling spacing


@pytest.mark.parametrize("name", ["c3lines", "c1round"])
def test_winding_matches_exact_membership(name):
    """Strong correctness (Section 1, O13.4): with round joins and caps the
    stroke is exactly {x : dist(x, path) <= w}.  Sampled points deeper than tau
    inside must have winding >= 1, points farther than tau outside winding 0,
    and no point has negative winding."""
    if name == "c1round":
        sc = S.scene_c1(1).subset([0, 1])
        sc.styles = sc.styles.copy()
        sc.styles["start_cap"] = S.CAP_ROUND
        sc.styles["end_cap"] = S.CAP_ROUND
        sc.styles["join"] = S.JOIN_ROUND
    else:
        sc = S.scene_c3(3, n_cubics=30, per_path=10, output_mode=S.OUT_LINES)
    r = O.expand(sc)
    tol = sc.tolerance
    rng = np.random.default_rng(3)
    for path in np.unique(r.out["path"]):
        o = r.out[r.out["path"] == path]
        v, pts = sc.path(int(path))
        w = float(sc.styles[sc.style_ix[path]]["half_width"])
        # dense source polyline of the path (FP64 from the FP32 input)
        src = []
        cur = None
        k = 0
        for verb in v:
            n = S.VERB_NPTS[int(verb)]
            q = pts[k : k + n].astype(np.float64)
            k += n
            if verb == S.MOVE:
                cur = q[0]
                start = cur
                continue
            if verb == S.CLOSE:
                q = start[None, :]
                verb = S.LINE
            ctrl = np.vstack([cur[None, :], q])
            if verb == S.LINE:
                P = np.array([ctrl[0], ctrl[0] + (ctrl[1] - ctrl[0]) / 3, ctrl[0] + 2 * (ctrl[1] - ctrl[0]) / 3, ctrl[1]])
            elif verb == S.QUAD:
                P = np.array([ctrl[0], ctrl[0] + 2 / 3 * (ctrl[1] - ctrl[0]), ctrl[2] + 2 / 3 * (ctrl[1] - ctrl[2]), ctrl[2]])
            else:
                P = ctrl
            src.append(X.dense_curve(P, 0.01)[1])
            cur = ctrl[-1]
        src = np.concatenate(src)
        tree = cKDTree(src)
        lo = src.min(0) - w - 3
        hi = src.max(0) + w + 3
        q = rng.uniform(lo, hi, (6000, 2))
        dist = tree.query(q)[0]
        wn = X.winding_numbers(o["x0"], o["y0"], o["x1"], o["y1"], q[:, 0], q[:, 1])
        assert np.all(wn >= 0)
        inside = dist < w - tol - 0.01
        outside = dist > w + tol + 0.01
        assert np.all(wn[inside] >= 1), (path, np.sum(wn[inside] < 1))
        assert np.all(wn[outside] == 0), (path, np.sum(wn[outside] != 0))


def test_evolutes_present_exactly_where_curvature_exceeds_reciprocal_width():
    sc = S.scene_c3(3, n_cubics=80, per_path=10, output_mode=S.OUT_LINES)
    r = O.expand(sc)
    offs = r.offsets()
    checked = 0
    for i, P, W, w in _segment_geometry(sc, r):
        o = r.out[offs[i] : offs[i + 1]]
        has_ev = np.any(o["kind"] == O.KIND_EVOLUTE)
        t = np.linspace(0, 1, 20001)
        d1 = X._bez_d(P, t)
        mt = 1 - t[:, None]
        d2 = 6 * (mt * (P[2] - 2 * P[1] + P[0]) + t[:, None] * (P[3] - 2 * P[2] + P[1]))
        cr = d1[:, 0] * d2[:, 1] - d1[:, 1] * d2[:, 0]
        sp = np.hypot(d1[:, 0], d1[:, 1])
        with np.errstate(divide="ignore", invalid="ignore"):
            kmax = np.nanmax(np.abs(cr) / sp**3)
        if kmax * w > 1.05:
            assert has_ev, i
            checked += 1
        elif kmax * w < 0.95:
            assert not has_ev, i
            checked += 1
    assert checked > 40


def test_round_join_points_lie_on_the_circle():
    sc = S.single_path_scene([0, 1, 1], [[0, 0], [100, 0], [30, 70]], 12.0, join=S.JOIN_ROUND, cap=S.CAP_BUTT)
    r = O.expand(sc)
    j = r.out[r.out["kind"] == O.KIND_JOIN_OUTER]
    assert len(j) > 3
    rad = np.hypot(np.r_[j["x0"], j["x1"]] - 100.0, np.r_[j["y0"], j["y1"]] - 0.0)
    assert np.max(np.abs(rad - 12.0)) < 1e-9
    # exact arc flattening (Section 2.1): each chord's sagitta <= tau_flat
    ang = np.abs(np.arctan2(j["y1"], j["x1"] - 100) - np.arctan2(j["y0"], j["x0"] - 100))
    ang = np.minimum(ang, 2 * math.pi - ang)
    assert np.all(12.0 * (1 - np.cos(ang / 2)) <= 0.65 * 0.25 + 1e-12)


def test_miter_limit_falls_back_to_bevel():
    # a 170 degree turn: miter ratio 1/cos(85 deg) = 11.5 > 4
    a = math.radians(170)
    sc = S.single_path_scene([0, 1, 1], [[0, 0], [100, 0], [100 + 50 * math.cos(a), 50 * math.sin(a)]], 5.0,
                             join=S.JOIN_MITER, cap=S.CAP_BUTT, miter_limit=4.0)
    r = O.expand(sc)
    assert np.sum(r.out["kind"] == O.KIND_JOIN_OUTER) == 1
    sc2 = S.single_path_scene([0, 1, 1], [[0, 0], [100, 0], [100 + 50 * math.cos(a), 50 * math.sin(a)]], 5.0,
                              join=S.JOIN_MITER, cap=S.CAP_BUTT, miter_limit=12.0)
    r2 = O.expand(sc2)
    assert np.sum(r2.out["kind"] == O.KIND_JOIN_OUTER) == 2


def test_paper_literal_fit_breaks_tolerance_for_wide_strokes():
    """Reading G2: with the paper's positional estimate alone (error = estimate x
    chord) the parallel curves of wide strokes leave the tolerance; the
    offset-aware reading keeps them inside."""
    sc = S.scene_c1(1).subset([1])
    worst = {}
    for fm in (O.FIT_PAPER, O.FIT_OFFSET):
        r = O.expand(sc, fit_mode=fm)
        offs = r.offsets()
        wmax = 0.0
        for i, P, W, w in _segment_geometry(sc, r):
            o = r.out[offs[i] : offs[i + 1]]
            o = o[o["kind"] == O.KIND_OFFSET]
            A, B, cusps = X.dense_offsets(P, w, 0.02)
            ref = np.concatenate([A, B] + [X.circle_pts(c, w) for c in cusps])
            pts, _ = X.sample_outputs(o["x0"], o["y0"], o["x1"], o["y1"], None, 0.05)
            wmax = max(wmax, X.max_dist(pts, ref)[0])
        worst[fm] = wmax
    assert worst[O.FIT_OFFSET] <= sc.tolerance
    assert worst[O.FIT_PAPER] > sc.tolerance
