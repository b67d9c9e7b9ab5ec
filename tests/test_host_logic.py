"""Host-side logic that needs no GPU: the autotuner's cache, the server's
admission and arrival process, the batch-scene generator."""
import json
import math
import os

import numpy as np
import pytest

from paper_2405_00127_amd import autotune as AT
from paper_2405_00127_amd import scenes as S
from paper_2405_00127_amd import serve as V


def test_workload_key_buckets_sizes_by_power_of_two():
    k1 = AT.workload_key("MI355X", 1_000_000, 0, 0.25)
    k2 = AT.workload_key("MI355X", 1_040_000, 0, 0.25)
    k3 = AT.workload_key("MI355X", 2_100_000, 0, 0.25)
    assert k1 == k2 != k3
    assert AT.workload_key("MI355X", 10, 1, 0.25) != AT.workload_key("MI355X", 10, 0, 0.25)
    assert AT.workload_key("MI355X", 10, 0, 0.1) != AT.workload_key("MI355X", 10, 0, 0.25)


def test_tuning_cache_roundtrip(tmp_path):
    path = str(tmp_path / "sub" / "tuning.json")
    assert AT._load(path) == {}
    AT._store(path, {"a": {"piece_waves": 2, "chunk_k": 16, "bisect_range": 256, "bisect_waves": 2}})
    assert AT._load(path)["a"]["chunk_k"] == 16
    with open(path, "w") as f:
        f.write("not json")
    assert AT._load(path) == {}


class _FakeCtx:
    """Records tuning calls; times come from a cost function (no GPU)."""

    device = 0

    def __init__(self, cost):
        self.t = {"piece_waves": 2, "chunk_k": 16, "bisect_range": 256, "bisect_waves": 2}
        self.cost = cost

    def set_tuning(self, **kw):
        self.t.update(kw)

    def get_tuning(self):
        return dict(self.t)


def test_tuner_picks_the_fastest_candidate(monkeypatch, tmp_path):
    def cost(t):  # separable: each group has one best value
        return (10.0 + abs(t["piece_waves"] - 1) + abs(t["bisect_range"] - 512) / 256 + abs(t["bisect_waves"] - 4)
                + abs(t["chunk_k"] - 32) / 8)

    ctx = _FakeCtx(cost)
    calls = []

    def fake_time(c, *a, **kw):
        calls.append(c.get_tuning())
        return c.cost(c.get_tuning())

    monkeypatch.setattr(AT, "time_config", fake_time)

    class _T:  # stands in for torch.cuda in the key
        class cuda:
            @staticmethod
            def current_stream():
                return None

            @staticmethod
            def get_device_name(d):
                return "fake"

    monkeypatch.setitem(__import__("sys").modules, "torch", _T)

    class _Scene:
        n_tags = 1000

    chosen, times = AT.tune(ctx, _Scene(), 0.25, 0, 0, 0, 0, stream=object(), cache_path=str(tmp_path / "t.json"))
    assert chosen == {"piece_waves": 1, "chunk_k": 32, "bisect_range": 512, "bisect_waves": 4}
    assert len(calls) == len(times)  # every candidate timed once
    # second call answers from the cache without timing anything
    ctx2 = _FakeCtx(cost)
    chosen2, times2 = AT.tune(ctx2, _Scene(), 0.25, 0, 0, 0, 0, stream=object(), cache_path=str(tmp_path / "t.json"))
    assert times2 == {} and chosen2 == chosen


def test_poisson_arrivals_rate():
    arr = V.poisson_arrivals(3, 1000.0, 20000)
    assert np.all(np.diff(arr) > 0)
    rate = len(arr) / arr[-1]
    assert abs(rate - 1000.0) / 1000.0 < 0.03


def test_admission_prediction_grows_with_observed_density():
    srv = V.Server.__new__(V.Server)
    srv.rec_per_seg = 0.0
    srv.rec_margin = 1.5
    r = V.Request(0, None, 1000, 0.0)
    p0 = srv._predict(r)
    assert p0 == int(1000 * 40.0 * 1.5) + 64
    srv.rec_per_seg = 12.0
    assert srv._predict(r) == int(1000 * 12.0 * 1.5) + 64


def test_batch_sizes_are_log_uniform_in_range():
    sz = S.batch_sizes(4, 256, 100, 200_000)
    assert sz.min() >= 100 and sz.max() < 200_000
    logs = np.log(sz)
    # log-uniform: the mean of log sizes sits mid-range
    mid = 0.5 * (math.log(100) + math.log(200_000))
    assert abs(logs.mean() - mid) < 0.5


def test_map_scene_structure():
    sc = S.scene_map(5, 3000, 30, 0.25, S.OUT_LINES)
    assert sc.n_segments() == 3000 and sc.n_paths == 30
    # every path starts with MOVE; per-verb point counts add up
    for k in range(sc.n_paths):
        v = sc.verbs[sc.verb_off[k]:sc.verb_off[k + 1]]
        assert v[0] == S.MOVE
        need = sum(S.VERB_NPTS[int(x)] for x in v)
        assert need == sc.pt_off[k + 1] - sc.pt_off[k]
    # points stay on the half-size canvas (placed by a x2 transform)
    assert sc.pts[:, 0].min() >= 0 and sc.pts[:, 0].max() <= S.CANVAS_W / 2 + 1e-3
    assert sc.pts[:, 1].min() >= 0 and sc.pts[:, 1].max() <= S.CANVAS_H / 2 + 1e-3
    kinds = sc.verbs[(sc.verbs >= S.LINE) & (sc.verbs <= S.CUBIC)]
    frac = np.bincount(kinds, minlength=4)[1:] / len(kinds)
    assert abs(frac[0] - 0.6) < 0.05 and abs(frac[1] - 0.15) < 0.05 and abs(frac[2] - 0.25) < 0.05
