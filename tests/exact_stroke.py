"""Independent FP64 checks of stroke outlines against the exact geometry.

Nothing here uses the method under test (no Euler spirals, no error
metrics, no subdivision counts).  The exact stroke boundary of a cubic
Bezier segment is its two parallel curves p(t) +/- w N(t), sampled densely
in FP64 (adaptive in t so that neighbouring samples are <= ``spacing``
apart), plus the exact join and cap shapes.  At an exact cusp the reference
is the near-cusp limit: the full circle of radius w about the cusp point.

These are test helpers only.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.spatial import cKDTree

TAG_COUNT, TAG_END, TAG_CLOSED = 0x03, 0x04, 0x80


def _bez(P, t):
    t = np.asarray(t, dtype=np.float64)[:, None]
    mt = 1.0 - t
    return mt**3 * P[0] + 3 * mt * mt * t * P[1] + 3 * mt * t * t * P[2] + t**3 * P[3]


def _bez_d(P, t):
    t = np.asarray(t, dtype=np.float64)[:, None]
    mt = 1.0 - t
    return 3 * (mt * mt * (P[1] - P[0]) + 2 * t * mt * (P[2] - P[1]) + t * t * (P[3] - P[2]))


def world_segment(data, monoid_off, tag, xf):
    """Elevated FP64 cubic of one encoded segment, in world space."""
    c = int(tag) & TAG_COUNT
    raw = data[monoid_off : monoid_off + c + 1].astype(np.float64)
    a, b, cc, d, e, f = [float(v) for v in xf]
    W = np.stack([a * raw[:, 0] + cc * raw[:, 1] + e, b * raw[:, 0] + d * raw[:, 1] + f], 1)
    if c == 1:
        P = np.array([W[0], W[0] + (W[1] - W[0]) / 3, W[0] + 2 * (W[1] - W[0]) / 3, W[1]])
    elif c == 2:
        P = np.array([W[0], W[0] + 2.0 / 3.0 * (W[1] - W[0]), W[2] + 2.0 / 3.0 * (W[1] - W[2]), W[2]])
    else:
        P = W.copy()
    return P, W


def end_tangents(W):
    """Direction of the curve leaving its start and arriving at its end."""
    c = len(W) - 1
    ts = next((W[j] - W[0] for j in range(1, c + 1) if np.any(W[j] != W[0])), np.array([1.0, 0.0]))
    te = next((W[c] - W[c - j] for j in range(1, c + 1) if np.any(W[c] != W[c - j])), np.array([1.0, 0.0]))
    return ts / np.linalg.norm(ts), te / np.linalg.norm(te)


def dense_curve(P, spacing=0.02, max_iter=12):
    """Adaptive t samples so that consecutive curve points are <= spacing apart
    (used for the source curve itself)."""
    t = np.linspace(0.0, 1.0, 257)
    for _ in range(max_iter):
        p = _bez(P, t)
        gap = np.hypot(*(p[1:] - p[:-1]).T)
        k = np.ceil(gap / spacing).astype(np.int64) - 1
        if not np.any(k > 0):
            break
        k = np.minimum(k, 4096)
        ins = [np.linspace(t[i], t[i + 1], k[i] + 2)[1:-1] for i in np.nonzero(k > 0)[0]]
        t = np.unique(np.concatenate([t] + ins))
    return t, _bez(P, t)


def dense_offsets(P, w, spacing=0.02, max_iter=40):
    """Dense FP64 samples of both parallel curves p +/- w N (N = right normal).

    Returns (A, B, cusps): point arrays for h = +w and h = -w, and a list of
    cusp points where the derivative vanishes (near-cusp limit circles)."""
    t = np.linspace(0.0, 1.0, 1025)
    cusps = []
    for it in range(max_iter):
        p = _bez(P, t)
        d = _bez_d(P, t)
        sp = np.hypot(d[:, 0], d[:, 1])
        with np.errstate(invalid="ignore", divide="ignore"):
            T = d / sp[:, None]
        N = np.stack([T[:, 1], -T[:, 0]], 1)
        A = p + w * N
        B = p - w * N
        good = np.isfinite(A).all(1)
        gap = np.maximum(np.hypot(*(A[1:] - A[:-1]).T), np.hypot(*(B[1:] - B[:-1]).T))
        gap = np.where(good[1:] & good[:-1], gap, np.inf)
        need = gap > spacing
        dtt = t[1:] - t[:-1]
        need &= dtt > 1e-13
        if not np.any(need):
            break
        k = np.where(need, np.minimum(np.ceil(np.minimum(gap, 1e9) / spacing), 64), 0).astype(np.int64) - 1
        k = np.maximum(k, np.where(need, 1, 0))
        ins = [np.linspace(t[i], t[i + 1], k[i] + 2)[1:-1] for i in np.nonzero(k > 0)[0]]
        t = np.unique(np.concatenate([t] + ins))
    p = _bez(P, t)
    d = _bez_d(P, t)
    sp = np.hypot(d[:, 0], d[:, 1])
    ok = sp > 0
    T = np.zeros_like(d)
    T[ok] = d[ok] / sp[ok, None]
    N = np.stack([T[:, 1], -T[:, 0]], 1)
    A = (p + w * N)[ok]
    B = (p - w * N)[ok]
    # remaining jumps larger than spacing at unresolvable t gaps are cusps
    gapA = np.hypot(*(A[1:] - A[:-1]).T)
    tt = t[ok]
    for i in np.nonzero((gapA > 4 * spacing) & ((tt[1:] - tt[:-1]) <= 1e-12))[0]:
        cusps.append(p[ok][i])
    # endpoints: use the end tangents of the control polygon (p1 == p0 etc.)
    return A, B, cusps


def circle_pts(c, r, a0=0.0, sweep=2 * math.pi, spacing=0.02):
    n = max(8, int(math.ceil(abs(sweep) * r / spacing)) + 1)
    a = a0 + np.linspace(0.0, sweep, n)
    return np.stack([c[0] + r * np.cos(a), c[1] + r * np.sin(a)], 1)


def line_pts(a, b, spacing=0.02):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    n = max(2, int(math.ceil(np.hypot(*(b - a)) / spacing)) + 1)
    s = np.linspace(0.0, 1.0, n)[:, None]
    return a + s * (b - a)


def sample_outputs(x0, y0, x1, y1, curv=None, spacing=0.05):
    """Dense points on output lines (curv == 0) or circular arcs."""
    pts = []
    idx = []
    for j in range(len(x0)):
        a = np.array([x0[j], y0[j]], np.float64)
        b = np.array([x1[j], y1[j]], np.float64)
        k = 0.0 if curv is None else float(curv[j])
        c = np.hypot(*(b - a))
        if k == 0.0 or c == 0.0 or abs(k) * c * c < 1e-12:
            # (a bulge c^2 |k| / 8 far below any tolerance: drawn as its chord,
            # which keeps the circle's centre from cancelling catastrophically)
            q = line_pts(a, b, spacing)
        else:
            # arc with chord a->b and signed curvature k (ccw positive)
            half = 0.5 * c * k
            half = max(-1.0, min(1.0, half))
            sweep = 2.0 * math.asin(half)  # signed turning
            r = 1.0 / abs(k)
            mid = 0.5 * (a + b)
            nrm = np.array([-(b - a)[1], (b - a)[0]]) / c  # left normal of chord
            dcen = math.sqrt(max(r * r - 0.25 * c * c, 0.0))
            cen = mid + nrm * dcen * (1 if k > 0 else -1)
            a0 = math.atan2(a[1] - cen[1], a[0] - cen[0])
            q = circle_pts(cen, r, a0, sweep, spacing)
        pts.append(q)
        idx.append(np.full(len(q), j))
    if not pts:
        return np.zeros((0, 2)), np.zeros(0, np.int64)
    return np.concatenate(pts), np.concatenate(idx)


def max_dist(points, ref, tree=None):
    if len(points) == 0:
        return 0.0, None
    if tree is None:
        tree = cKDTree(ref)
    d, _ = tree.query(points)
    j = int(np.argmax(d))
    return float(d[j]), j


def winding_numbers(x0, y0, x1, y1, qx, qy):
    """Nonzero winding number of a line soup at query points (exact for lines;
    arcs should be flattened by the caller)."""
    w = np.zeros(len(qx), dtype=np.int64)
    for a in range(0, len(x0), 4096):
        X0 = x0[a : a + 4096][None, :]
        Y0 = y0[a : a + 4096][None, :]
        X1 = x1[a : a + 4096][None, :]
        Y1 = y1[a : a + 4096][None, :]
        px = qx[:, None]
        py = qy[:, None]
        up = (Y0 <= py) & (Y1 > py)
        dn = (Y1 <= py) & (Y0 > py)
        cr = (X1 - X0) * (py - Y0) - (px - X0) * (Y1 - Y0)
        w += np.sum(up & (cr > 0), axis=1) - np.sum(dn & (cr < 0), axis=1)
    return w


def flatten_arcs(out_x0, out_y0, out_x1, out_y1, curv, spacing=0.05):
    pts, idx = sample_outputs(out_x0, out_y0, out_x1, out_y1, curv, spacing)
    # consecutive samples of the same output form lines
    same = idx[1:] == idx[:-1]
    a = pts[:-1][same]
    b = pts[1:][same]
    return a[:, 0], a[:, 1], b[:, 0], b[:, 1]
