"""GPU-vs-oracle comparison with the decision-margin exclusions.

Rules (per tag):
  * monoids, encoding: bit-exact (checked elsewhere);
  * record counts identical, except for tags where one of the oracle's
    decisions sits within a threshold of its boundary (fit error vs tau_fit,
    a count estimate vs an integer, a rho sign, the cusp perturbation test,
    the hodograph test, a join classification) -- FP32 and FP64 may
    legitimately decide those differently;
  * for tags with equal counts: every record's endpoints within ENDPOINT_TOL
    px, arcs' bulge (midpoint distance from the chord) within SWEEP_TOL px,
    path ids equal.
"""
from __future__ import annotations

import dataclasses

import numpy as np

ENDPOINT_TOL = 1e-3
SWEEP_TOL = 1e-3  # px, arc bulge
# Margin thresholds.  Both sides take every decision in FP64 (the GPU from
# the same FP32 inputs, evaluating the curve relative to the segment start),
# so only decisions within ~1e-9 (relative; absolute for count estimates and
# the unit-tangent cross product) of their threshold may legitimately differ.
FIT_MARGIN = 1e-9
COUNT_MARGIN = 1e-9
RHO_MARGIN = 1e-9
Q_MARGIN = 1e-9
HODO_MARGIN = 1e-9
JOIN_MARGIN = 1e-12


@dataclasses.dataclass
class ParityReport:
    n_tags: int
    n_near: int
    n_count_mismatch: int
    n_unexplained: int
    n_compared_records: int
    worst_endpoint: float
    worst_sweep: float
    worst_tag: int
    bad_path_ids: int

    def ok(self):
        return (self.n_unexplained == 0 and self.worst_endpoint <= ENDPOINT_TOL and self.worst_sweep <= SWEEP_TOL
                and self.bad_path_ids == 0)


def arc_bulge(recs) -> np.ndarray:
    """Signed distance from an arc record's chord midpoint to the arc,
    (c/2) tan(sweep/4) with sin(sweep/2) = curvature c / 2."""
    x0 = recs["x0"].astype(np.float64)
    c = np.hypot(recs["x1"].astype(np.float64) - x0, recs["y1"].astype(np.float64) - recs["y0"])
    half = np.clip(recs["curv"].astype(np.float64) * c / 2.0, -1.0, 1.0)
    sweep = 2.0 * np.arcsin(half)
    return c / 2.0 * np.tan(sweep / 4.0)


def near_threshold(margins) -> np.ndarray:
    m = margins
    return ((m["fit"] < FIT_MARGIN) | (m["count"] < COUNT_MARGIN) | (m["rho"] < RHO_MARGIN) |
            (m["q"] < Q_MARGIN) | (m["len"] < HODO_MARGIN) | (m["join"] < JOIN_MARGIN))


def compare(gpu_counts, gpu_recs, ref, mode, tags=None) -> ParityReport:
    """gpu_counts: u32 per tag (all tags); gpu_recs: structured numpy records
    of the whole output; ref: oracle Result over the same tags (all of them,
    or the subset ``tags`` when the oracle ran tag-by-tag)."""
    gc = np.asarray(gpu_counts, dtype=np.int64)
    go = np.concatenate([[0], np.cumsum(gc)])
    oc = ref.counts.astype(np.int64)
    oo = np.concatenate([[0], np.cumsum(oc)])
    if tags is None:
        tags = np.arange(len(gc))
    near = near_threshold(ref.margins)
    mism = gc[tags] != oc[tags]
    unexplained = mism & ~near[tags]
    # geometry is compared where the counts agree and no decision was close
    same_tags = tags[~mism & ~near[tags]]
    # gather matched records
    lens = gc[same_tags]
    tot = int(lens.sum())
    worst_e = worst_s = 0.0
    worst_tag = -1
    bad_ids = 0
    if tot:
        rep = np.repeat(np.arange(len(same_tags)), lens)
        within = np.arange(tot) - np.repeat(np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
        gi = go[same_tags][rep] + within
        oi = oo[same_tags][rep] + within
        g = gpu_recs[gi]
        r = ref.out[oi]
        d = np.max(np.abs(np.stack([g["x0"] - r["x0"], g["y0"] - r["y0"], g["x1"] - r["x1"], g["y1"] - r["y1"]])), axis=0)
        j = int(np.argmax(d))
        worst_e = float(d[j])
        worst_tag = int(same_tags[rep[j]])
        if mode == 1:
            worst_s = float(np.max(np.abs(arc_bulge(g) - arc_bulge(r))))
        bad_ids = int(np.sum(g["path"] != r["path"]))
    return ParityReport(len(tags), int(near[tags].sum()), int(mism.sum()), int(unexplained.sum()), tot, worst_e,
                        worst_s, worst_tag, bad_ids)


def closed_per_path(recs) -> int:
    """Number of paths whose start-point multiset differs from the end-point
    multiset (bit-exact)."""
    bad = 0
    order = np.argsort(recs["path"], kind="stable")
    r = recs[order]
    cut = np.nonzero(np.diff(r["path"]))[0] + 1
    for grp in np.split(r, cut):
        s = np.sort(np.stack([grp["x0"].view(np.uint32), grp["y0"].view(np.uint32)], 1).view(np.uint64).ravel())
        e = np.sort(np.stack([grp["x1"].view(np.uint32), grp["y1"].view(np.uint32)], 1).view(np.uint64).ravel())
        if not np.array_equal(s, e):
            bad += 1
    return bad
