"""The exact-density mode (SX_DENSITY_NEWTON: line counts from the exact
subdivision density integral, points by the f_approx inverse refined with two
Newton steps; Section 4.2) against the oracle's same mode, through the C ABI,
at the parity bars of the default mode."""
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
    c = B.Context(0, density=B.DENSITY_NEWTON)
    assert c.config()["density"] == B.DENSITY_NEWTON
    yield c
    c.close()


@pytest.mark.parametrize("name", ["c1_lines", "c2_lines", "c3_lines", "c1_arcs"])
def test_newton_mode_parity(ctx, name):
    import torch

    from paper_2405_00127_amd import binding as B

    sc = {"c1_lines": lambda: S.scene_c1(1),
          "c2_lines": lambda: S.scene_c2(2, n_segments=40000, n_paths=400),
          "c3_lines": lambda: S.scene_c3(3, n_cubics=3000, output_mode=S.OUT_LINES),
          "c1_arcs": lambda: S.scene_c1(1, output_mode=S.OUT_ARCS)}[name]()
    _say("newton parity", name)
    mode = sc.output_mode
    scene = ctx.encode(sc)
    recs, n, _ = ctx.expand(scene, sc.tolerance, mode)
    counts = ctx.counts(scene, sc.tolerance, mode).cpu().numpy().astype(np.uint32)
    torch.cuda.synchronize()
    got = B.records_to_numpy(recs, mode)
    ref = O.expand(sc, fit_mode=O.DENSITY_NEWTON)
    rep = P.compare(counts, got, ref, mode)
    _say(name, rep)
    assert rep.ok(), rep
    assert rep.n_count_mismatch <= max(3, 0.01 * rep.n_tags), rep
    assert P.closed_per_path(got) == 0
    if mode == S.OUT_ARCS:
        # arcs are placed uniformly in arc length (Section 5): the mode changes nothing
        assert np.array_equal(ref.counts, O.expand(sc, emit=False).counts)
    scene.release()


def test_newton_mode_full_map_scene(ctx):
    """The 1M-segment map scene with lines in the exact-density mode: counts
    of every tag against the oracle and the records of sampled tags."""
    import torch

    from paper_2405_00127_amd import binding as B

    sc = S.scene_c2(2)
    _say("newton full c2")
    scene = ctx.encode(sc)
    recs, n, _ = ctx.expand(scene, sc.tolerance, sc.output_mode)
    counts = ctx.counts(scene).cpu().numpy().astype(np.uint32)
    torch.cuda.synchronize()
    got = B.records_to_numpy(recs, sc.output_mode)
    ref = O.expand(sc, emit=False, fit_mode=O.DENSITY_NEWTON)
    near = P.near_threshold(ref.margins)
    mism = counts != ref.counts
    _say("newton full c2: tags", len(counts), "records", n, "mismatch", int(mism.sum()), "near", int(near.sum()))
    assert not np.any(mism & ~near)
    go = np.concatenate([[0], np.cumsum(counts.astype(np.int64))])
    rng = np.random.default_rng(4)
    worst = 0.0
    for i in np.sort(rng.choice(np.nonzero(~mism)[0], 1500, replace=False)):
        r = O.expand(sc, emit=True, tag_begin=int(i), tag_end=int(i) + 1, enc=ref.enc, fit_mode=O.DENSITY_NEWTON,
                     margins=False)
        g = got[go[i]:go[i + 1]]
        o = r.out
        assert len(o) == len(g)
        if len(g):
            d = max(np.max(np.abs(g["x0"] - o["x0"])), np.max(np.abs(g["y0"] - o["y0"])),
                    np.max(np.abs(g["x1"] - o["x1"])), np.max(np.abs(g["y1"] - o["y1"])))
            worst = max(worst, float(d))
    _say("newton full c2: sampled worst endpoint", worst)
    assert worst <= P.ENDPOINT_TOL
    assert P.closed_per_path(got) == 0
    scene.release()
