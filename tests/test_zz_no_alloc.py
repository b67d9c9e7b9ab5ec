"""The allocation-free scan (sx_scan_u32_noalloc, its scratch in a static
device array) against sx_scan_u32 (which allocates its scratch per call),
through the C ABI: bit-exact on two calls in a row, the second smaller, then
larger again; empty input; the size limit rejected without a launch."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


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


def test_noalloc_scan_matches_the_allocating_scan(ctx):
    import torch

    from paper_2405_00127_amd import binding as B

    rng = np.random.default_rng(17)
    for n in [3_000_017, 70_001, 8192 * 5 + 1, 1, 4_100_000]:
        _say("noalloc scan n =", n)
        v = rng.integers(0, 3000, n).astype(np.uint32)
        t = torch.from_numpy(v.view(np.int32)).cuda()
        want = ctx.scan_u32(t)
        out = torch.full((n + 1,), -1, dtype=torch.int64, device="cuda")
        got = ctx.scan_u32_noalloc(t, out)
        torch.cuda.synchronize()
        assert torch.equal(got, want), n
        assert int(got[-1]) == int(v.astype(np.uint64).sum())


def test_noalloc_scan_edge_sizes(ctx):
    import torch

    from paper_2405_00127_amd import binding as B

    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    out = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    ctx.scan_u32_noalloc(e, out)
    torch.cuda.synchronize()
    assert int(out[0]) == 0
    big = B.lib().sx_scan_u32_noalloc
    import ctypes as C

    rc = big(C.c_void_p(ctx.h), C.c_void_p(out.data_ptr()), C.c_void_p(out.data_ptr()), (1 << 24) + 1, None)
    assert rc == B.SX_EINVAL
    # still usable afterwards
    v = torch.arange(1000, dtype=torch.int32, device="cuda")
    assert torch.equal(ctx.scan_u32_noalloc(v), ctx.scan_u32(v))
