"""Pins of the oracle's dashing (the dashed encoding of readings G34-G36,
then the ordinary expansion) against hand-derived dashes, the exact arc
length, circles and the exact stroke of the dashes.  CPU only."""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.spatial import cKDTree

import exact_stroke as X
import oracle as O
from paper_2405_00127_amd import scenes as S

TAG_END, TAG_CLOSED, TAG_PATH = 0x04, 0x80, 0x10


def _line_scene(pattern, offset, cap=S.CAP_BUTT, w=2.0, pts=((0, 0), (100, 0)), verbs=None):
    verbs = verbs or [S.MOVE] + [S.LINE] * (len(pts) - 1)
    sc = S.single_path_scene(verbs, list(pts), w, join=S.JOIN_MITER, cap=cap)
    sc.dashes = [(np.asarray(pattern, np.float32), float(offset))]
    return sc


def _rects(r):
    return np.round(np.stack([r.out["x0"], r.out["y0"], r.out["x1"], r.out["y1"]], 1), 9)


@pytest.mark.parametrize("pattern,offset,dashes", [
    ([10, 5], 0.0, [(0, 10), (15, 25), (30, 40), (45, 55), (60, 70), (75, 85), (90, 100)]),
    ([10, 5], 3.0, [(0, 7), (12, 22), (27, 37), (42, 52), (57, 67), (72, 82), (87, 97)]),
    ([10, 5], -4.0, [(4, 14), (19, 29), (34, 44), (49, 59), (64, 74), (79, 89), (94, 100)]),  # offset -4 = 11
    ([30], 0.0, [(0, 30), (60, 90)]),          # an odd array repeats: 30 on, 30 off
    ([20, 10, 5, 10], 0.0, [(0, 20), (30, 35), (45, 65), (75, 80), (90, 100)]),
])
def test_dashed_line_is_exact_rectangles(pattern, offset, dashes):
    """A horizontal line of length 100, half-width 2, butt caps: each dash
    [a, b] is exactly the rectangle [a, b] x [-2, 2] (two offset lines and
    two caps), in order."""
    r = O.expand(_line_scene(pattern, offset), enc=O.encode_dashed(_line_scene(pattern, offset)))
    assert r.status == 0
    got = _rects(r)
    want = []
    for a, b in dashes:
        want += [[a, -2, b, -2], [b, 2, a, 2], [b, -2, b, 2], [a, 2, a, -2]]
    assert got.shape == (len(want), 4)
    assert np.max(np.abs(got - np.array(want, float))) < 1e-9


def test_dash_spanning_a_corner_keeps_its_join():
    """A right-angle polyline (0,0)-(50,0)-(50,50) with dashes of 20 every
    35: the dash over the corner ([35, 55] along the path) is one open
    subpath with a miter join at (50, 0); the others are straight."""
    sc = _line_scene([20, 15], 0.0, pts=((0, 0), (50, 0), (50, 50)))
    enc = O.encode_dashed(sc)
    r = O.expand(sc, enc=enc)
    assert r.status == 0
    joins = r.out[(r.out["kind"] == O.KIND_JOIN_OUTER) | (r.out["kind"] == O.KIND_JOIN_INNER)]
    assert len(joins) == 4  # the miter's two lines and the inner pivot's two lines
    # the miter point of a right angle with half-width 2
    pts = np.concatenate([np.stack([joins["x0"], joins["y0"]], 1), np.stack([joins["x1"], joins["y1"]], 1)])
    assert np.min(np.hypot(pts[:, 0] - 52.0, pts[:, 1] + 2.0)) < 1e-9
    # dashes [0, 20], [35, 55] and [70, 90] = 20..40 up the second segment
    markers = np.nonzero((enc.tags & TAG_END) != 0)[0]
    assert len(markers) == 2 + 3  # the two empty path markers and one per dash
    caps = r.out[r.out["kind"] == O.KIND_CAP]
    assert len(caps) == 6


def test_closed_subpath_dashes_are_open_and_split_at_the_start():
    """A closed square of side 40 (perimeter 160) with dashes of 50 every 80
    and offset 20: the dash that would run over the start point is cut there
    into [0, 30] and [140, 160]; no dash is closed."""
    sc = S.single_path_scene([S.MOVE, S.LINE, S.LINE, S.LINE, S.CLOSE], [[0, 0], [40, 0], [40, 40], [0, 40]], 1.0,
                             join=S.JOIN_MITER, cap=S.CAP_BUTT)
    sc.dashes = [(np.array([50, 30], np.float32), 20.0)]
    enc = O.encode_dashed(sc)
    markers = np.nonzero((enc.tags & TAG_END) != 0)[0]
    inner = markers[1:-1]
    assert len(inner) == 3  # [0,30], [60,110], [140,160]
    assert np.all((enc.tags[inner] & TAG_CLOSED) == 0)
    assert np.all((enc.tags[markers[[0, -1]]] & TAG_CLOSED) != 0)
    r = O.expand(sc, enc=enc)
    caps = r.out[r.out["kind"] == O.KIND_CAP]
    assert len(caps) == 6


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_arc_length_rule_against_adaptive_quadrature(seed):
    """Reading G35's 16-panel Gauss-Legendre arc length against the exact
    arc length (adaptive quadrature of |B'|): within 1e-9 relative where the
    speed stays above a tenth of its maximum, within 1e-4 relative on any
    cubic, near and at exact cusps included (where |B'| has a kink)."""
    rng = np.random.default_rng(seed)
    for k in range(60):
        P = rng.uniform(0, 200, (4, 2))
        if k % 4 == 3:
            # an exact cusp: a (p1 - p0) + b (p2 - p1) + c (p3 - p2) = 0 at tc
            tc = rng.uniform(0.2, 0.8)
            a, b, c = (1 - tc) ** 2, 2 * tc * (1 - tc), tc * tc
            P[2] = (a * (P[1] - P[0]) - b * P[1] + c * P[3]) / (c - b)

        def speed(t):
            return np.hypot(*(3 * ((1 - t) ** 2 * (P[1] - P[0]) + 2 * t * (1 - t) * (P[2] - P[1])
                                   + t * t * (P[3] - P[2]))))
        true = integrate.quad(speed, 0, 1, epsabs=0, epsrel=1e-13, limit=400)[0]
        sp = np.array([speed(t) for t in np.linspace(0, 1, 2001)])
        smooth = sp.min() > 0.1 * sp.max()
        err = abs(O.dash_seg_len(P) / true - 1)
        assert err < (1e-9 if smooth else 1e-4), (k, err, sp.min() / sp.max())


def test_dashes_on_a_circle_land_at_their_arc_lengths():
    """Four cubics approximating a circle of radius 100 (the 4/3 tan rule),
    dashes of 20 every 30 (length units): every dash start and end point lies
    on the circle (within the cubics' own deviation from it) at the angle
    arc length / radius, to within 1e-3 rad."""
    R = 100.0
    k = 4.0 / 3.0 * math.tan(math.pi / 8)
    pts = [[R, 0]]
    for q in range(4):
        a0, a1 = q * math.pi / 2, (q + 1) * math.pi / 2
        p0 = np.array([math.cos(a0), math.sin(a0)]) * R
        p3 = np.array([math.cos(a1), math.sin(a1)]) * R
        t0 = np.array([-math.sin(a0), math.cos(a0)])
        t1 = np.array([-math.sin(a1), math.cos(a1)])
        pts += [list(p0 + k * R * t0), list(p3 - k * R * t1), list(p3)]
    sc = S.single_path_scene([S.MOVE] + [S.CUBIC] * 4, pts, 1.0, join=S.JOIN_ROUND, cap=S.CAP_BUTT)
    sc.dashes = [(np.array([20, 10], np.float32), 0.0)]
    enc = O.encode_dashed(sc)
    mon = O.monoids(enc.tags)
    ends = []
    for i in np.nonzero((enc.tags & TAG_END) != 0)[0][1:-1]:
        ends.append(enc.data[mon[0][i] + 1])  # the dash's start point (marker)
        ends.append(enc.data[mon[0][i]])      # the dash's last point
    ends = np.array(ends, np.float64)
    rad = np.hypot(ends[:, 0], ends[:, 1])
    assert np.max(np.abs(rad - R)) < 0.03  # the 4/3 tan cubics stay within 2.7e-4 R
    ang = np.mod(np.arctan2(ends[:, 1], ends[:, 0]), 2 * math.pi)
    perim = 2 * math.pi * R
    want = []
    for m in range(int(perim // 30) + 1):
        a, b = 30 * m, min(30 * m + 20, perim)
        if a < perim:
            want += [a / R, b / R]
    want = np.array(want)
    # pair each measured angle with the nearest expected one
    err = np.min(np.abs(ang[:, None] - want[None, :]), axis=1)
    err = np.minimum(err, 2 * math.pi - err)
    assert np.max(err) < 1e-3


def test_dashed_outlines_follow_the_exact_dash_strokes():
    """Random cubic paths with dash patterns: every offset output within tau
    of the exact parallel curves of its dash part, every output closed per
    path, and with round joins and caps the winding number equals exact
    membership in the union of the dashes' strokes (points within w of a
    dash part)."""
    sc = S.with_dashes(S.scene_c1(1).subset(range(2)), seed=5, lo=4.0, hi=40.0)
    sc.styles = sc.styles.copy()
    sc.styles["join"] = S.JOIN_ROUND
    sc.styles["start_cap"] = S.CAP_ROUND
    sc.styles["end_cap"] = S.CAP_ROUND
    enc = O.encode_dashed(sc)
    r = O.expand(sc, enc=enc)
    assert r.status == 0
    mon = O.monoids(enc.tags)
    offs = r.offsets()
    tol = sc.tolerance
    worst = 0.0
    parts_by_path = {}
    for i in np.nonzero((enc.tags & TAG_END) == 0)[0]:
        xf = sc.xforms[enc.xform_stream[mon[3][i]]]
        w = float(sc.styles[enc.style_stream[mon[2][i]]]["half_width"])
        P, W = X.world_segment(enc.data, mon[0][i], enc.tags[i], xf)
        o = r.out[offs[i]: offs[i + 1]]
        o = o[o["kind"] == O.KIND_OFFSET]
        A, B, cusps = X.dense_offsets(P, w, 0.02)
        ref = np.concatenate([A, B] + [X.circle_pts(c, w) for c in cusps])
        pts, _ = X.sample_outputs(o["x0"], o["y0"], o["x1"], o["y1"], None, 0.05)
        worst = max(worst, X.max_dist(pts, ref)[0])
        parts_by_path.setdefault(int(enc.path_map[mon[1][i]]), []).append((X.dense_curve(P, 0.01)[1], w))
    assert worst <= tol
    rng = np.random.default_rng(2)
    for path, parts in parts_by_path.items():
        o = r.out[r.out["path"] == path]
        w = parts[0][1]
        src = np.concatenate([p for p, _ in parts])
        lo, hi = src.min(0) - w - 3, src.max(0) + w + 3
        q = rng.uniform(lo, hi, (3000, 2))
        dist = cKDTree(src).query(q)[0]
        wn = X.winding_numbers(o["x0"], o["y0"], o["x1"], o["y1"], q[:, 0], q[:, 1])
        assert np.all(wn >= 0)
        assert np.all(wn[dist < w - tol - 0.01] >= 1)
        assert np.all(wn[dist > w + tol + 0.01] == 0)


def test_solid_and_filled_paths_are_copied():
    """Paths without a pattern (and fills, which are never dashed) keep
    their tags and points; only the two empty subpaths per path are added."""
    sc = S.with_fills(S.scene_c1(1).subset(range(4)), 0.5, seed=3)
    sc.dashes = None
    enc = O.encode(sc)
    de = O.encode_dashed(sc, enc=enc)
    keep = np.ones(len(de.tags), bool)
    m = np.nonzero((de.tags & TAG_END) != 0)[0]
    empty = m[(de.tags[m] & TAG_CLOSED) != 0]
    # drop the added empty subpaths (those whose marker follows another marker or starts the stream)
    added = [k for k in empty if k == 0 or (de.tags[k - 1] & TAG_END)]
    keep[added] = False
    assert len(added) == 2 * sc.n_paths
    body = de.tags[keep]
    src = enc.tags & ~np.uint8(TAG_PATH | 0x40 | 0x20)
    assert np.array_equal(body, src)
    assert np.array_equal(de.style_stream, enc.style_stream)
    assert np.array_equal(de.path_map, enc.path_map)


def _dash_structure(enc):
    """(segments without extent, open subpaths without segments) of an
    encoding: a segment has extent when one of its points differs from its
    start point."""
    mon = O.monoids(enc.tags)
    flat, empty_open = 0, 0
    for i, t in enumerate(enc.tags):
        if t & TAG_END:
            if not (t & TAG_CLOSED) and (i == 0 or (enc.tags[i - 1] & TAG_END)):
                empty_open += 1
            continue
        c = int(t & 3)
        D = enc.data[mon[0][i] : mon[0][i] + c + 1]
        if np.all(D[1:] == D[0]):
            flat += 1
    return flat, empty_open


def test_dash_starting_a_fraction_of_an_ulp_before_a_segment_end():
    """Reading G36's rule for parts without extent.  The polyline
    (1000,0)-(1010,0)-(1010,10) with dashes of 5 every 10 and offset 2^-20:
    the second dash starts 2^-20 before the corner, where x = 1010 - 2^-20
    rounds to 1010 in FP32, so its part of the first segment has no extent.
    That part is left out: the dash is the vertical stretch from (1010, 0)
    to (1010, 5 - 2^-20), its cap marker points along +y, and with butt caps
    its outline is exactly the rectangle [1008, 1012] x [0, 5 - 2^-20] (no
    join at the corner, no undefined tangents)."""
    sc = _line_scene([5, 5], 2.0 ** -20, pts=((1000, 0), (1010, 0), (1010, 10)))
    enc = O.encode_dashed(sc)
    assert _dash_structure(enc) == (0, 0)
    mon = O.monoids(enc.tags)
    markers = [i for i, t in enumerate(enc.tags) if (t & TAG_END) and not (t & TAG_CLOSED)]
    # dashes: [0, 5 - 2^-20), [10 - 2^-20, 15 - 2^-20), [20 - 2^-20, 20)
    assert len(markers) == 3
    m2 = enc.data[mon[0][markers[1]] + 1 : mon[0][markers[1]] + 3]  # (the point before is the last point)
    assert m2[0].tolist() == [1010.0, 0.0]
    assert m2[1][0] == 1010.0 and m2[1][1] > 4.9
    r = O.expand(sc, enc=enc)
    assert r.status == 0
    o = r.out
    xy = np.stack([o["x0"], o["y0"], o["x1"], o["y1"]], 1)
    assert np.all(np.isfinite(xy))
    second = o[(np.minimum(o["x0"], o["x1"]) >= 1007.9) & (np.maximum(o["y0"], o["y1"]) <= 5.5)]
    assert len(second) == 4 and len(r.out[(r.out["kind"] == O.KIND_JOIN_OUTER)]) == 0
    ys = np.concatenate([second["y0"], second["y1"]])
    xs = np.concatenate([second["x0"], second["x1"]])
    assert abs(ys.min() - 0.0) < 1e-9 and abs(ys.max() - (5 - 2.0 ** -20)) < 1e-5
    assert abs(xs.min() - 1008.0) < 1e-9 and abs(xs.max() - 1012.0) < 1e-9


def test_dashes_shorter_than_an_ulp_draw_nothing():
    """Dashes of 2^-20 units every 1 + 2^-20 along a segment at x ~ 1000,
    where the FP32 spacing is 2^-16: most dashes round to a single point and
    draw nothing; those that straddle a rounding boundary remain as tiny
    dashes with extent.  No segment of the encoding lacks extent and no dash
    is empty."""
    sc = _line_scene([2.0 ** -20, 1.0], 0.0, pts=((1000, 0), (1010, 0)))
    enc = O.encode_dashed(sc)
    assert _dash_structure(enc) == (0, 0)
    n_dash = int(np.count_nonzero(((enc.tags & TAG_END) != 0) & ((enc.tags & TAG_CLOSED) == 0)))
    assert n_dash <= 3
    r = O.expand(sc, enc=enc)
    assert r.status == 0 and np.all(np.isfinite(r.out["x0"]))


@pytest.mark.parametrize("name", ["c1", "map", "stress"])
def test_dashed_encodings_have_no_parts_without_extent(name):
    """Every segment of a dashed encoding has extent and every dash has a
    segment, on seeded scenes whose dash boundaries fall anywhere."""
    sc = {"c1": lambda: S.with_dashes(S.scene_c1(1), seed=1),
          "map": lambda: S.with_dashes(S.scene_c2(2, n_segments=20000, n_paths=200), seed=4, lo=0.5, hi=12.0),
          "stress": lambda: S.with_dashes(S.scene_c3(3, n_cubics=500), seed=6, lo=2.0, hi=30.0)}[name]()
    enc = O.encode_dashed(sc)
    assert enc.status == 0
    assert _dash_structure(enc) == (0, 0)
