"""Seeded synthetic scene generators.

These produce *input* paths only (verbs, control points, styles, transforms).
Nothing here implements any step of the stroke-expansion method: no encoding,
no tangents, no subdivision, no offsetting.  Both the HIP path and the FP64
oracle consume the same generated scenes.

The paper's datasets (Nehab's *timings*, mmark, long dash) are not available,
so these recipes stand in for them with the shapes the paper describes: map /
CAD scenes of many paths with millions of segments (Section 1), random
line/quad/cubic strokes in the style of the MotionMark canvas-paths test
(Section 9.2), and cusp / loop stress cubics (Section 7.3).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# Path verbs (SVG commands, Section 8.1).
MOVE, LINE, QUAD, CUBIC, CLOSE = 0, 1, 2, 3, 4
VERB_NPTS = {MOVE: 1, LINE: 1, QUAD: 2, CUBIC: 3, CLOSE: 0}

# Join / cap / output enums (SVG stroke styles, Section 8 criteria).
JOIN_BEVEL, JOIN_MITER, JOIN_ROUND = 0, 1, 2
CAP_BUTT, CAP_SQUARE, CAP_ROUND = 0, 1, 2
OUT_LINES, OUT_ARCS = 0, 1

STYLE_DTYPE = np.dtype(
    [
        ("half_width", "<f4"),
        ("miter_limit", "<f4"),
        ("join", "u1"),
        ("start_cap", "u1"),
        ("end_cap", "u1"),
        ("flags", "u1"),
    ],
    align=False,
)
assert STYLE_DTYPE.itemsize == 12

CANVAS_W, CANVAS_H = 2088.0, 1600.0

# Style flag bit 0: the path is filled (flattened at offset 0), not stroked.
STYLE_FILL = 1


@dataclasses.dataclass
class Scene:
    """A batch of paths in a flat, C-friendly layout.

    verbs     u8  [n_verbs]       all paths' verbs, path after path
    verb_off  u32 [n_paths + 1]   path k owns verbs[verb_off[k]:verb_off[k+1]]
    pts       f32 [n_pts, 2]      all control points, path after path
    pt_off    u32 [n_paths + 1]   path k owns pts[pt_off[k]:pt_off[k+1]]
    style_ix  u32 [n_paths]       index into ``styles``
    xform_ix  u32 [n_paths]       index into ``xforms``
    styles    STYLE_DTYPE [n_styles]
    xforms    f32 [n_xforms, 6]   (a, b, c, d, e, f): x' = a x + c y + e, y' = b x + d y + f
    dashes    optional, one entry per style: None (solid) or (dash lengths,
              dash offset) in the path's own units (SVG dasharray/dashoffset)
    """

    verbs: np.ndarray
    verb_off: np.ndarray
    pts: np.ndarray
    pt_off: np.ndarray
    style_ix: np.ndarray
    xform_ix: np.ndarray
    styles: np.ndarray
    xforms: np.ndarray
    name: str = ""
    tolerance: float = 0.25
    output_mode: int = OUT_LINES
    dashes: Optional[list] = None

    @property
    def n_paths(self) -> int:
        return int(len(self.verb_off) - 1)

    def n_segments(self) -> int:
        """Number of LINE/QUAD/CUBIC verbs (input segments, before closing lines)."""
        v = self.verbs
        return int(np.count_nonzero((v == LINE) | (v == QUAD) | (v == CUBIC)))

    def path(self, k: int):
        v = self.verbs[self.verb_off[k] : self.verb_off[k + 1]]
        p = self.pts[self.pt_off[k] : self.pt_off[k + 1]]
        return v, p

    def subset(self, path_ids) -> "Scene":
        """A scene made of the given paths (styles / transforms kept whole)."""
        b = SceneBuilder()
        for k in path_ids:
            v, p = self.path(int(k))
            b.add_path(v, p, int(self.style_ix[k]), int(self.xform_ix[k]))
        sc = b.build(self.styles, self.xforms, name=self.name + "[subset]",
                     tolerance=self.tolerance, output_mode=self.output_mode)
        sc.dashes = self.dashes
        return sc

    def dash_tables(self):
        """The dash patterns as flat arrays: values (f32), per-style offsets
        into them (u32, n_styles + 1) and dash offsets (f32, n_styles)."""
        n = len(self.styles)
        ds = self.dashes or [None] * n
        vals, off, ph = [], [0], []
        for k in range(n):
            d = ds[k] if k < len(ds) else None
            arr, o = (d if d is not None else ((), 0.0))
            vals.extend(float(v) for v in arr)
            off.append(len(vals))
            ph.append(float(o))
        return (np.asarray(vals, np.float32), np.asarray(off, np.uint32), np.asarray(ph, np.float32))


class SceneBuilder:
    def __init__(self):
        self._verbs: List[np.ndarray] = []
        self._pts: List[np.ndarray] = []
        self._style: List[int] = []
        self._xform: List[int] = []

    def add_path(self, verbs, pts, style_ix: int, xform_ix: int = 0):
        verbs = np.asarray(verbs, dtype=np.uint8)
        pts = np.asarray(pts, dtype=np.float32).reshape(-1, 2)
        need = sum(VERB_NPTS[int(v)] for v in verbs)
        if need != len(pts):
            raise ValueError(f"path needs {need} points, got {len(pts)}")
        self._verbs.append(verbs)
        self._pts.append(pts)
        self._style.append(style_ix)
        self._xform.append(xform_ix)

    def build(self, styles, xforms=None, name="", tolerance=0.25, output_mode=OUT_LINES) -> Scene:
        if xforms is None:
            xforms = identity_xforms()
        nv = np.array([len(v) for v in self._verbs], dtype=np.int64)
        npt = np.array([len(p) for p in self._pts], dtype=np.int64)
        verb_off = np.zeros(len(nv) + 1, dtype=np.uint32)
        pt_off = np.zeros(len(npt) + 1, dtype=np.uint32)
        verb_off[1:] = np.cumsum(nv)
        pt_off[1:] = np.cumsum(npt)
        verbs = np.concatenate(self._verbs) if self._verbs else np.zeros(0, np.uint8)
        pts = np.concatenate(self._pts) if self._pts else np.zeros((0, 2), np.float32)
        return Scene(
            verbs=np.ascontiguousarray(verbs, dtype=np.uint8),
            verb_off=verb_off,
            pts=np.ascontiguousarray(pts, dtype=np.float32),
            pt_off=pt_off,
            style_ix=np.asarray(self._style, dtype=np.uint32),
            xform_ix=np.asarray(self._xform, dtype=np.uint32),
            styles=np.ascontiguousarray(styles, dtype=STYLE_DTYPE),
            xforms=np.ascontiguousarray(np.asarray(xforms, dtype=np.float32).reshape(-1, 6)),
            name=name,
            tolerance=float(tolerance),
            output_mode=int(output_mode),
        )


def identity_xforms() -> np.ndarray:
    return np.array([[1, 0, 0, 1, 0, 0]], dtype=np.float32)


def make_styles(half_width, join, start_cap, end_cap=None, miter_limit=4.0) -> np.ndarray:
    half_width = np.atleast_1d(np.asarray(half_width, dtype=np.float32))
    n = len(half_width)
    s = np.zeros(n, dtype=STYLE_DTYPE)
    s["half_width"] = half_width
    s["miter_limit"] = np.broadcast_to(np.asarray(miter_limit, np.float32), (n,))
    s["join"] = np.broadcast_to(np.asarray(join, np.uint8), (n,))
    s["start_cap"] = np.broadcast_to(np.asarray(start_cap, np.uint8), (n,))
    if end_cap is None:
        end_cap = start_cap
    s["end_cap"] = np.broadcast_to(np.asarray(end_cap, np.uint8), (n,))
    return s


def single_path_scene(verbs, pts, half_width, join=JOIN_ROUND, cap=CAP_ROUND,
                      miter_limit=4.0, tolerance=0.25, output_mode=OUT_LINES,
                      xform=None, end_cap=None) -> Scene:
    b = SceneBuilder()
    b.add_path(verbs, pts, 0, 0)
    xf = identity_xforms() if xform is None else np.asarray(xform, np.float32).reshape(1, 6)
    return b.build(make_styles([half_width], join, cap, end_cap, miter_limit), xf,
                   name="single", tolerance=tolerance, output_mode=output_mode)


def _dir(a):
    return np.array([math.cos(a), math.sin(a)])


# --------------------------------------------------------------------------
# Config 1: 50 paths / 1,000 cubics in a 1024 px box.
# --------------------------------------------------------------------------
def scene_c1(seed: int = 1, n_paths: int = 50, n_cubics: int = 1000,
             box: float = 1024.0, tolerance: float = 0.25,
             output_mode: int = OUT_LINES) -> Scene:
    """Uniform control points, 50% tangent-continuous joints, half the paths
    closed, half-width U(1, 20), round joins, butt caps."""
    rng = np.random.Generator(np.random.PCG64(seed))
    # multinomial split, every path gets at least one cubic
    counts = 1 + rng.multinomial(n_cubics - n_paths, np.full(n_paths, 1.0 / n_paths))
    closed = rng.random(n_paths) < 0.5
    widths = rng.uniform(1.0, 20.0, n_paths).astype(np.float32)
    b = SceneBuilder()
    for k in range(n_paths):
        n = int(counts[k])
        p0 = rng.uniform(0, box, 2)
        pts = [p0]
        verbs = [MOVE]
        prev_p2 = None
        cur = p0
        for j in range(n):
            p1 = rng.uniform(0, box, 2)
            if prev_p2 is not None and rng.random() < 0.5:
                lam = rng.uniform(0.5, 2.0)
                p1 = cur + lam * (cur - prev_p2)
            p2 = rng.uniform(0, box, 2)
            p3 = rng.uniform(0, box, 2)
            verbs.append(CUBIC)
            pts += [p1, p2, p3]
            prev_p2, cur = p2, p3
        if closed[k]:
            verbs.append(CLOSE)
        b.add_path(verbs, np.array(pts), k, 0)
    styles = make_styles(widths, JOIN_ROUND, CAP_BUTT)
    return b.build(styles, name=f"c1-seed{seed}", tolerance=tolerance, output_mode=output_mode)


# --------------------------------------------------------------------------
# Config 2 / 4 / 5: map / CAD shaped scenes.
# --------------------------------------------------------------------------
def _path_lengths(rng, n_paths: int, total: int, lo: float = 2.0, hi: float = 2000.0) -> np.ndarray:
    raw = np.exp(rng.uniform(math.log(lo), math.log(hi), n_paths))
    if n_paths * 2 > total:
        raise ValueError("total too small for the path count")
    scaled = raw * (total / raw.sum())
    lens = np.maximum(2, np.floor(scaled)).astype(np.int64)
    # fix the sum exactly: distribute the remainder over the largest fractional parts
    diff = total - int(lens.sum())
    if diff > 0:
        frac = scaled - np.floor(scaled)
        order = np.argsort(-frac)
        i = 0
        while diff > 0:
            lens[order[i % n_paths]] += 1
            diff -= 1
            i += 1
    elif diff < 0:
        order = np.argsort(-lens)
        i = 0
        while diff < 0:
            j = order[i % n_paths]
            if lens[j] > 2:
                lens[j] -= 1
                diff += 1
            i += 1
    assert int(lens.sum()) == total
    return lens


def scene_map(seed: int = 2, n_segments: int = 1_000_000, n_paths: Optional[int] = None,
              tolerance: float = 0.25, output_mode: int = OUT_LINES,
              scale: float = 2.0) -> Scene:
    """Map / CAD shaped scene.

    * path lengths log-uniform in [2, 2000], rescaled to sum to ``n_segments``;
    * each path is a random walk on the 2088x1600 canvas; chord length
      lognormal (median 6 px, sigma 0.8) clipped to [0.25, 400]; heading
      change N(0, 0.6 rad) except at 50% tangent-continuous joints;
    * segment kinds i.i.d.: 60% lines, 15% quads, 25% cubics; curve control
      arms at angles U(-1, 1) rad from the chord with lengths U(0.1, 0.6) of it;
    * half-width lognormal (median 1.5 px, sigma 1.0) clipped to [0.05, 50];
    * joins uniform over miter (limit 4) / round / bevel, caps uniform over
      butt / square / round, 30% of paths closed.

    Geometry is generated in a half-size local frame and placed on the
    canvas by a uniform-scale transform (the paper scales its scenes up by
    encoding a transform, Section 9.2).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if n_paths is None:
        n_paths = max(1, n_segments // 100)
    lens = _path_lengths(rng, n_paths, n_segments)
    widths = np.clip(np.exp(rng.normal(math.log(1.5), 1.0, n_paths)), 0.05, 50.0)
    joins = rng.integers(0, 3, n_paths)  # 0 bevel, 1 miter, 2 round
    caps = rng.integers(0, 3, n_paths)
    closed = rng.random(n_paths) < 0.3
    styles = make_styles((widths / scale).astype(np.float32), joins.astype(np.uint8),
                         caps.astype(np.uint8), caps.astype(np.uint8), 4.0)
    W, H = CANVAS_W / scale, CANVAS_H / scale
    total = int(lens.sum())
    # draw all randomness for all segments at once (vectorised), then walk
    kind_u = rng.random(total)
    kinds = np.where(kind_u < 0.6, LINE, np.where(kind_u < 0.75, QUAD, CUBIC)).astype(np.uint8)
    chord = np.clip(np.exp(rng.normal(math.log(6.0), 0.8, total)), 0.25, 400.0) / scale
    g1 = rng.random(total) < 0.5
    dturn = rng.normal(0.0, 0.6, total)
    th_a = rng.uniform(-1.0, 1.0, total)
    th_b = rng.uniform(-1.0, 1.0, total)
    arm_a = rng.uniform(0.1, 0.6, total)
    arm_b = rng.uniform(0.1, 0.6, total)
    starts = np.stack([rng.uniform(0, W, n_paths), rng.uniform(0, H, n_paths)], 1)
    heads = rng.uniform(-math.pi, math.pi, n_paths)

    # layout: path k = MOVE, its segments, CLOSE if closed; a segment of kind
    # LINE / QUAD / CUBIC carries 1 / 2 / 3 points (the verb codes)
    seg_start = np.zeros(n_paths + 1, dtype=np.int64)
    np.cumsum(lens, out=seg_start[1:])
    pc = kinds.astype(np.int64)
    path_of_seg = np.repeat(np.arange(n_paths), lens)
    cum_pc = np.zeros(total + 1, dtype=np.int64)
    np.cumsum(pc, out=cum_pc[1:])
    pts_per_path = 1 + (cum_pc[seg_start[1:]] - cum_pc[seg_start[:-1]])
    verbs_per_path = 1 + lens + closed.astype(np.int64)
    pt_off = np.zeros(n_paths + 1, dtype=np.int64)
    np.cumsum(pts_per_path, out=pt_off[1:])
    verb_off = np.zeros(n_paths + 1, dtype=np.int64)
    np.cumsum(verbs_per_path, out=verb_off[1:])
    # first point of each segment in the point stream, its verb slot
    seg_pt = pt_off[path_of_seg] + 1 + (cum_pc[:-1] - cum_pc[seg_start[path_of_seg]])
    seg_verb = verb_off[path_of_seg] + 1 + (np.arange(total) - seg_start[path_of_seg])
    verbs_all = np.empty(int(verb_off[-1]), dtype=np.uint8)
    pts_all = np.empty((int(pt_off[-1]), 2), dtype=np.float64)
    verbs_all[verb_off[:-1]] = MOVE
    verbs_all[seg_verb] = kinds
    verbs_all[verb_off[1:][closed] - 1] = CLOSE
    pts_all[pt_off[:-1]] = starts

    def unit(a):
        return np.stack([np.cos(a), np.sin(a)], 1)

    # the walks of all paths advance together, one segment per step
    cur = starts.copy()
    tan = heads.copy()
    for j in range(int(lens.max()) if n_paths else 0):
        K = np.nonzero(lens > j)[0]
        si = seg_start[K] + j
        st = np.where(g1[si] & (j > 0), tan[K], tan[K] + dturn[si])
        kind = kinds[si]
        L = chord[si]
        cdir = np.where(kind == LINE, st, st - th_a[si])
        c0 = cur[K]
        end = c0 + L[:, None] * unit(cdir)
        # reflect the walk at the canvas borders
        rx = ~((end[:, 0] >= 0.0) & (end[:, 0] <= W))
        cdir = np.where(rx, math.pi - cdir, cdir)
        st = np.where(rx, math.pi - st, st)
        ry = ~((end[:, 1] >= 0.0) & (end[:, 1] <= H))
        cdir = np.where(ry, -cdir, cdir)
        st = np.where(ry, -st, st)
        end = c0 + L[:, None] * unit(cdir)
        end = np.clip(end, 0.0, [W, H])
        base = seg_pt[si]
        new_tan = cdir.copy()
        m = kind == LINE
        pts_all[base[m]] = end[m]
        m = kind == QUAD
        if m.any():
            # control point along the start tangent
            c1 = c0[m] + (arm_a[si[m]] * L[m])[:, None] * unit(st[m]) * 1.5
            pts_all[base[m]] = c1
            pts_all[base[m] + 1] = end[m]
            d = end[m] - c1
            nz = (d[:, 0] != 0.0) | (d[:, 1] != 0.0)
            new_tan[m] = np.where(nz, np.arctan2(d[:, 1], d[:, 0]), cdir[m])
        m = kind == CUBIC
        if m.any():
            et = cdir[m] + th_b[si[m]]
            c1 = c0[m] + (arm_a[si[m]] * L[m])[:, None] * unit(st[m])
            c2 = end[m] - (arm_b[si[m]] * L[m])[:, None] * unit(et)
            pts_all[base[m]] = c1
            pts_all[base[m] + 1] = c2
            pts_all[base[m] + 2] = end[m]
            new_tan[m] = et
        tan[K] = new_tan
        cur[K] = end
    vi = int(verb_off[-1])
    pi = int(pt_off[-1])
    verb_off = verb_off.astype(np.uint32)
    pt_off = pt_off.astype(np.uint32)
    xf = np.array([[scale, 0, 0, scale, 0, 0]], dtype=np.float32)
    return Scene(
        verbs=verbs_all[:vi].copy(),
        verb_off=verb_off,
        pts=pts_all[:pi].astype(np.float32),
        pt_off=pt_off,
        style_ix=np.arange(n_paths, dtype=np.uint32),
        xform_ix=np.zeros(n_paths, dtype=np.uint32),
        styles=styles,
        xforms=xf,
        name=f"map-{n_segments}-seed{seed}",
        tolerance=tolerance,
        output_mode=output_mode,
    )


def with_fills(scene: Scene, frac: float = 1.0, seed: int = 0, xform=None) -> Scene:
    """A copy of ``scene`` in which a seeded fraction ``frac`` of the styles
    are fills (every path drawn with such a style is flattened at offset 0
    and closed).  With ``xform`` (six floats, any invertible affine map), the
    fill paths are drawn with that transform appended to the table."""
    rng = np.random.default_rng(seed)
    styles = scene.styles.copy()
    n = len(styles)
    pick = rng.random(n) < frac if frac < 1.0 else np.ones(n, bool)
    styles["flags"] = np.where(pick, styles["flags"] | STYLE_FILL, styles["flags"])
    xforms = scene.xforms
    xform_ix = scene.xform_ix
    if xform is not None:
        xforms = np.concatenate([xforms, np.asarray(xform, np.float32).reshape(1, 6)])
        fill_path = pick[scene.style_ix]
        xform_ix = np.where(fill_path, len(xforms) - 1, scene.xform_ix).astype(np.uint32)
    return dataclasses.replace(scene, styles=styles, xforms=np.ascontiguousarray(xforms, np.float32),
                               xform_ix=np.ascontiguousarray(xform_ix, np.uint32),
                               name=scene.name + f"-fill{frac:g}")


def scene_c2(seed: int = 2, output_mode: int = OUT_LINES, n_segments: int = 1_000_000,
             n_paths: int = 10_000) -> Scene:
    return scene_map(seed, n_segments, n_paths, 0.25, output_mode)


# --------------------------------------------------------------------------
# Config 3: strong-correctness stress cubics.
# --------------------------------------------------------------------------
def _cubic_eval_d(p, t):
    """Derivative of a cubic Bezier (used only to build test geometry)."""
    p0, p1, p2, p3 = p
    mt = 1 - t
    return 3 * (mt * mt * (p1 - p0) + 2 * t * mt * (p2 - p1) + t * t * (p3 - p2))


def _cusp_p2(p0, p1, p3, tc):
    # solve B'(tc) = 0 for p2 (linear); singular at tc = 2/3
    mt = 1 - tc
    rhs = -(mt * mt) * (p1 - p0) + 2 * tc * mt * p1 - tc * tc * p3
    return rhs / (tc * (2 - 3 * tc))


_PAIRS = {}


def _pair_block(m, i0):
    """Index pairs (i, j) with i in [i0, i0 + 64) and j >= i + 2, j < m."""
    key = (m, i0)
    if key not in _PAIRS:
        i, j = np.nonzero(np.arange(m)[None, :] >= np.arange(i0, min(i0 + 64, m - 2))[:, None] + 2)
        _PAIRS[key] = (i + i0, j)
    return _PAIRS[key]


def _self_intersects(p, n=257):
    t = np.linspace(0, 1, n)[:, None]
    mt = 1 - t
    q = mt**3 * p[0] + 3 * mt * mt * t * p[1] + 3 * mt * t * t * p[2] + t**3 * p[3]
    a = q[:-1]
    b = q[1:]
    d1 = b - a
    m = len(a)
    # brute force over the non-adjacent segment pairs (i, j >= i + 2), a
    # block of rows i at a time, middle rows first (a loop's crossing pairs an
    # early segment with a late one); stops at the first block with a crossing
    for i0 in (64, 0, 128, 192):
        if i0 >= m - 2:
            continue
        i, j = _pair_block(m, i0)
        o = a[j]
        e = b[j] - o
        den = d1[i, 0] * e[:, 1] - d1[i, 1] * e[:, 0]
        w = o - a[i]
        with np.errstate(divide="ignore", invalid="ignore"):
            s = (w[:, 0] * e[:, 1] - w[:, 1] * e[:, 0]) / den
            u = (w[:, 0] * d1[i, 1] - w[:, 1] * d1[i, 0]) / den
        if np.any((den != 0) & (s >= 0) & (s <= 1) & (u >= 0) & (u <= 1)):
            return True
    return False


_CURV_T = np.linspace(0, 1, 4097)


def _max_curv_fp64(cubics):
    """FP64 maximum curvature of each cubic (array [n, 4, 2]) over 4097
    parameter samples."""
    t = _CURV_T[None, :, None]
    mt = 1 - t
    p = cubics[:, None, :, :]
    d1 = 3 * (mt * mt * (p[:, :, 1] - p[:, :, 0]) + 2 * t * mt * (p[:, :, 2] - p[:, :, 1])
              + t * t * (p[:, :, 3] - p[:, :, 2]))
    d2 = 6 * (mt * (p[:, :, 2] - 2 * p[:, :, 1] + p[:, :, 0]) + t * (p[:, :, 3] - 2 * p[:, :, 2] + p[:, :, 1]))
    cr = d1[..., 0] * d2[..., 1] - d1[..., 1] * d2[..., 0]
    sp = np.hypot(d1[..., 0], d1[..., 1])
    with np.errstate(divide="ignore", invalid="ignore"):
        k = np.abs(cr) / sp**3
    k[~np.isfinite(k)] = np.inf
    return np.max(k, axis=1)


def stress_cubic(rng, kind: int) -> np.ndarray:
    """One stress cubic in a local frame with p0 at the origin, chord ~U(10,100)."""
    L = rng.uniform(10.0, 100.0)
    while True:
        if kind in (0, 1):  # exact / near cusp
            p0 = np.zeros(2)
            p3 = np.array([L, 0.0])
            p1 = np.array([rng.uniform(-0.5, 1.5) * L, rng.uniform(-1.0, 1.0) * L])
            while True:
                tc = rng.uniform(0.1, 0.9)
                if abs(tc - 2.0 / 3.0) > 0.05:
                    break
            p2 = _cusp_p2(p0, p1, p3, tc)
            if np.max(np.abs(p2)) > 4 * L:
                continue
            if kind == 1:
                mag = 10.0 ** rng.uniform(-4.0, 0.0)
                p2 = p2 + mag * _dir(rng.uniform(-math.pi, math.pi))
            pts = np.array([p0, p1, p2, p3])
        elif kind == 2:  # self loop: crossed arms
            hgt = rng.uniform(0.4, 1.5) * L * (1 if rng.random() < 0.5 else -1)
            p1 = np.array([rng.uniform(1.0, 1.6) * L, hgt])
            p2 = np.array([rng.uniform(-0.6, 0.0) * L, hgt * rng.uniform(0.7, 1.3)])
            pts = np.array([[0.0, 0.0], p1, p2, [L, 0.0]])
            if not _self_intersects(pts):
                continue
        else:  # degenerate control polygons
            sub = rng.integers(0, 4)
            a = np.array([rng.uniform(0.2, 0.8) * L, rng.uniform(-0.5, 0.5) * L])
            if sub == 0:  # p1 == p0
                pts = np.array([[0.0, 0.0], [0.0, 0.0], a, [L, 0.0]])
            elif sub == 1:  # p2 == p3
                pts = np.array([[0.0, 0.0], a, [L, 0.0], [L, 0.0]])
            elif sub == 2:  # p1 == p2
                pts = np.array([[0.0, 0.0], a, a, [L, 0.0]])
            else:  # collinear, backtracking beyond the end point
                pts = np.array([[0.0, 0.0], [1.6 * L, 0.0], [-0.4 * L, 0.0], [L, 0.0]])
        return pts


def scene_c3(seed: int = 3, n_cubics: int = 100_000, per_path: int = 10,
             tolerance: float = 0.1, output_mode: int = OUT_ARCS,
             min_frac_over: float = 0.4) -> Scene:
    """Cusp / near-cusp / self-loop / degenerate cubics, 25% each, chained
    into open paths; half-widths U(5, 50) px; at least ``min_frac_over`` of
    segments have FP64 max curvature * half-width > 1."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_paths = max(1, n_cubics // per_path)
    for attempt in range(20):
        widths = rng.uniform(5.0, 50.0, n_paths)
        b = SceneBuilder()
        all_c32 = []
        for k in range(n_paths):
            cur = np.array([rng.uniform(0, CANVAS_W), rng.uniform(0, CANVAS_H)])
            verbs = [MOVE]
            pts = [cur.copy()]
            for j in range(per_path):
                kind = int(rng.integers(0, 4))
                c = stress_cubic(rng, kind)
                ang = rng.uniform(-math.pi, math.pi)
                R = np.array([[math.cos(ang), -math.sin(ang)], [math.sin(ang), math.cos(ang)]])
                c = c @ R.T + cur
                all_c32.append(c.astype(np.float32).astype(np.float64))
                verbs.append(CUBIC)
                pts += [c[1], c[2], c[3]]
                cur = c[3]
            b.add_path(verbs, np.array(pts), k, 0)
        # count segments with max curvature x half-width > 1 (stops once
        # enough are found)
        cubics = np.array(all_c32)
        wseg = np.repeat(widths, per_path)
        need = min_frac_over * n_paths * per_path
        over = 0
        for c in range(0, len(cubics), 256):
            over += int(np.count_nonzero(_max_curv_fp64(cubics[c:c + 256]) * wseg[c:c + 256] > 1.0))
            if over >= need:
                break
        if over >= need:
            break
    styles = make_styles(widths.astype(np.float32), JOIN_ROUND, CAP_ROUND)
    return b.build(styles, name=f"c3-seed{seed}", tolerance=tolerance, output_mode=output_mode)


# --------------------------------------------------------------------------
# Config 4 / 5: many scenes of uneven size.
# --------------------------------------------------------------------------
def batch_sizes(seed: int, n: int, lo: int, hi: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), n))).astype(np.int64)


def scene_batch(seed: int = 4, n_scenes: int = 256, lo: int = 100, hi: int = 200_000,
                output_mode: int = OUT_LINES) -> List[Scene]:
    sizes = batch_sizes(seed, n_scenes, lo, hi)
    out = []
    for i, s in enumerate(sizes):
        s = int(max(s, 4))
        out.append(scene_map(seed * 100_003 + i, s, max(1, s // 100), 0.25, output_mode))
    return out


def with_dashes(scene: Scene, seed: int = 0, lo: float = 1.0, hi: float = 24.0, max_len: int = 4) -> Scene:
    """The scene with a seeded dash pattern on every stroke style: 1..max_len
    (dash, gap) pairs of lengths log-uniform in [lo, hi] (in the path's own
    units) and an offset uniform in one period; fills stay solid."""
    rng = np.random.Generator(np.random.PCG64(seed))
    dashes = []
    for st in scene.styles:
        if int(st["flags"]) & STYLE_FILL:
            dashes.append(None)
            continue
        m = 2 * int(rng.integers(1, max_len + 1))
        arr = np.exp(rng.uniform(math.log(lo), math.log(hi), m)).astype(np.float32)
        dashes.append((arr, float(rng.uniform(0.0, float(arr.sum())))))
    out = dataclasses.replace(scene, name=scene.name + "-dashed")
    out.dashes = dashes
    return out
