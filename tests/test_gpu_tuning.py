"""Launch parameters never change the outline (GPU, through the C ABI).

The autotuner picks, per workload, the piece launch's waves per SIMD (the
template instantiation of the slot kernel), the bisection's waves per SIMD
and tags per wave, and the records per item chunk of the record kernel.
Every instantiation the tuner can pick is run here on the full-size map
scene (lines and arcs) and the full-size stress scene; the records must be
bit-identical to those of the default launch parameters, which the parity
tests compare with the oracle.  C1 is compared with the oracle directly at
every one of them.  The paper-literal fit mode of the context configuration
is compared with the oracle's paper-literal mode."""
import sys

import numpy as np
import pytest

import oracle as O
import parity as P
from paper_2405_00127_amd import scenes as S

pytestmark = pytest.mark.gpu

# (piece_waves, chunk_k, bisect_range, bisect_waves): every slot-kernel and
# bisection instantiation, chunk sizes and ranges across the tuner's grid,
# including the committed tunings of the 1M-segment map scene (lines and
# arcs (1, 16, 192, 4)) and of the 256-scene batch (2, 16, 512, 2)
GRID = [(2, 16, 256, 2), (1, 4, 1024, 2), (2, 8, 128, 3), (3, 32, 128, 4), (3, 16, 192, 3), (3, 64, 384, 2),
        (1, 32, 256, 4), (3, 4, 128, 2), (1, 16, 192, 4), (2, 16, 512, 2)]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    from paper_2405_00127_amd import binding as B

    torch.cuda.set_device(0)
    c = B.Context(0)
    yield c
    c.close()


def _run(ctx, scene, tol, mode, tuning):
    import torch

    ctx.set_tuning(*tuning)
    recs, n, buf = ctx.expand(scene, tol, mode)
    torch.cuda.synchronize()
    return n, buf


@pytest.mark.parametrize("name", ["c2_lines", "c2_arcs", "c3_arcs"])
def test_every_tuning_gives_identical_records(ctx, name):
    import torch

    sc = {"c2_lines": lambda: S.scene_c2(2), "c2_arcs": lambda: S.scene_c2(2, output_mode=S.OUT_ARCS),
          "c3_arcs": lambda: S.scene_c3(3)}[name]()
    _say("tuning grid", name, sc.n_segments(), "segments")
    scene = ctx.encode(sc)
    rec = 24 if sc.output_mode == S.OUT_ARCS else 20
    n0, ref = _run(ctx, scene, sc.tolerance, sc.output_mode, GRID[0])
    ref = ref[: n0 * rec].clone()
    try:
        for t in GRID[1:]:
            n, buf = _run(ctx, scene, sc.tolerance, sc.output_mode, t)
            _say("  tuning", t, "records", n)
            assert n == n0, t
            assert torch.equal(buf[: n * rec], ref), t
    finally:
        ctx.set_tuning(*GRID[0])


@pytest.mark.parametrize("mode", [S.OUT_LINES, S.OUT_ARCS])
def test_c1_parity_at_every_tuning(ctx, mode):
    from paper_2405_00127_amd import binding as B

    sc = S.scene_c1(1, output_mode=mode)
    ref = O.expand(sc)
    scene = ctx.encode(sc)
    try:
        for t in GRID:
            ctx.set_tuning(*t)
            recs, n, _ = ctx.expand(scene, sc.tolerance, mode)
            counts = ctx.counts(scene, sc.tolerance, mode).cpu().numpy().astype(np.uint32)
            rep = P.compare(counts, B.records_to_numpy(recs, mode), ref, mode)
            _say("c1", mode, t, rep)
            assert rep.ok(), (t, rep)
    finally:
        ctx.set_tuning(*GRID[0])


@pytest.mark.parametrize("mode", [S.OUT_LINES, S.OUT_ARCS])
def test_paper_literal_fit_mode_matches_the_oracle(mode):
    """SX_FIT_PAPER (the Section 7.1 estimate times the chord, without the
    width term) against the oracle's paper-literal mode: same parity bars."""
    import torch

    from paper_2405_00127_amd import binding as B

    sc = S.scene_c1(1, output_mode=mode)
    c = B.Context(0, fit_mode=B.FIT_PAPER)
    try:
        assert c.config()["fit_mode"] == B.FIT_PAPER
        scene = c.encode(sc)
        recs, n, _ = c.expand(scene, sc.tolerance, mode)
        counts = c.counts(scene, sc.tolerance, mode).cpu().numpy().astype(np.uint32)
        torch.cuda.synchronize()
        ref = O.expand(sc, fit_mode=O.FIT_PAPER)
        rep = P.compare(counts, B.records_to_numpy(recs, mode), ref, mode)
        _say("paper fit", mode, rep)
        assert rep.ok(), rep
        assert P.closed_per_path(B.records_to_numpy(recs, mode)) == 0
        scene.release()
    finally:
        c.close()


def test_bad_configuration_is_rejected():
    from paper_2405_00127_amd import binding as B

    for kw in ({"fit_mode": 2}, {"density": 7}):
        with pytest.raises(B.StrokexError) as ei:
            B.Context(0, **kw)
        assert ei.value.code == B.SX_EINVAL
