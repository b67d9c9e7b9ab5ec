"""Continuous-batching server: every request's outline is the same, bit for
bit, as the scene expanded alone, whatever it was batched with; the
overflow path (output arena or item workspace too small) re-runs a batch and
still returns the same records."""
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


def _pool(ctx, mode):
    scs = [S.scene_map(40 + i, n, max(1, n // 100), 0.25, mode) for i, n in enumerate([120, 4000, 900, 25000, 60])]
    scs.append(S.scene_c3(3, n_cubics=80))
    return scs, [ctx.encode(sc) for sc in scs]


def _alone(ctx, scene, tol, mode):
    from paper_2405_00127_amd import binding as B

    recs, n, _ = ctx.expand(scene, tol, mode)
    return B.records_to_numpy(recs, mode).copy()


@pytest.mark.parametrize("mode,budget", [(S.OUT_LINES, 60_000_000), (S.OUT_ARCS, 50_000), (S.OUT_LINES, 1_000)])
def test_server_results_equal_alone(ctx, mode, budget):
    import time

    from paper_2405_00127_amd import binding as B
    from paper_2405_00127_amd import serve as V

    tol = 0.25
    scs, pool = _pool(ctx, mode)
    _say("serve, mode", mode, "record budget", budget)
    alone = [_alone(ctx, s, tol, mode) for s in pool]
    rng = np.random.Generator(np.random.PCG64(9))
    picks = rng.integers(0, len(pool), 40)
    checked = {}

    def on_done(r, recs):
        # runs before the request's slot takes new work
        got = B.records_to_numpy(recs, mode)
        k = int(picks[r.rid])
        checked[r.rid] = np.array_equal(got.view(np.uint8), alone[k].view(np.uint8))

    srv = V.Server(ctx, tol, mode, n_slots=2, seg_budget=30_000, rec_budget=budget, max_batch=8, on_done=on_done)
    t0 = time.perf_counter()
    for i, k in enumerate(picks):
        srv.submit(V.Request(i, pool[k], scs[k].n_segments(), time.perf_counter()))
        if i % 5 == 4:  # requests keep arriving while batches run
            srv.step(time.perf_counter())
    while srv.busy() and time.perf_counter() < t0 + 60.0:
        srv.step(time.perf_counter())
    assert not srv.busy()
    assert len(checked) == len(picks)
    bad = [rid for rid, ok in checked.items() if not ok]
    assert not bad, bad
    assert srv.batches > 1
    if budget < 10_000:
        assert sum(sl.reruns for sl in srv.slots) > 0
    srv.close()


def test_server_lone_request_on_a_fresh_scene(ctx):
    """A request taken alone runs as a plain expansion of its scene; on a
    scene never expanded before, its item workspace starts small, so the slot
    sizes it and re-runs; the records equal the scene expanded alone."""
    import time

    from paper_2405_00127_amd import binding as B
    from paper_2405_00127_amd import serve as V

    tol, mode = 0.25, S.OUT_LINES
    sc = S.scene_map(77, 30000, 300, tol, mode)
    got = {}

    def on_done(r, recs):
        got[r.rid] = B.records_to_numpy(recs, mode).copy()

    srv = V.Server(ctx, tol, mode, n_slots=1, rec_budget=1_000, on_done=on_done)
    srv.submit(V.Request(0, ctx.encode(sc), sc.n_segments(), 0.0))
    t0 = time.perf_counter()
    while srv.busy() and time.perf_counter() < t0 + 60.0:
        srv.step(0.0)
    assert not srv.busy()
    assert srv.batches == 1 and srv.slots[0].reruns >= 1
    ref = _alone(ctx, ctx.encode(sc), tol, mode)
    assert np.array_equal(got[0].view(np.uint8), ref.view(np.uint8))
    srv.close()
