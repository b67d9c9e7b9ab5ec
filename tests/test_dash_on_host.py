"""The dashing passes' device code (dash_len_d, dash_tag) built for the host
and driven serially, against the oracle's dashed encoding: the same tags bit
for bit and the same points (FP32; a point may differ by one ulp where the
two sides' FP64 parameters round differently).  CPU only."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_2405_00127_amd import scenes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_00127_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")


class _Paths(C.Structure):
    _fields_ = [("verbs", C.c_void_p), ("verb_off", C.c_void_p), ("pts", C.c_void_p), ("pt_off", C.c_void_p),
                ("style_ix", C.c_void_p), ("xform_ix", C.c_void_p), ("n_paths", C.c_uint32)]


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if not HIPCC:
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("dashhost") / "libdashhost.so")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-shared",
                           "-ffp-contract=off", "-Wno-unused-command-line-argument",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", out,
                           os.path.join(os.path.dirname(__file__), "host", "dash_on_host.hip"),
                           os.path.join(CSRC, "sx_encode.cpp")], stderr=subprocess.DEVNULL)
    L = C.CDLL(out)
    L.dh_dash.argtypes = [C.POINTER(_Paths), C.c_void_p, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint32,
                          C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint64, C.POINTER(C.c_uint64),
                          C.POINTER(C.c_uint64)]
    return L


def dash_host(L, sc):
    keep = [np.ascontiguousarray(sc.verbs, np.uint8), np.ascontiguousarray(sc.verb_off, np.uint32),
            np.ascontiguousarray(sc.pts, np.float32), np.ascontiguousarray(sc.pt_off, np.uint32),
            np.ascontiguousarray(sc.style_ix, np.uint32), np.ascontiguousarray(sc.xform_ix, np.uint32)]
    p = _Paths(*[k.ctypes.data for k in keep], sc.n_paths)
    st = np.ascontiguousarray(sc.styles)
    vals, off, ph = sc.dash_tables()
    vals = np.ascontiguousarray(vals if len(vals) else np.zeros(1, np.float32))
    nt, npt = C.c_uint64(), C.c_uint64()
    args = (C.byref(p), st.ctypes.data, len(st), vals.ctypes.data, off.ctypes.data, ph.ctypes.data, len(sc.xforms))
    assert L.dh_dash(*args, None, None, 0, 0, C.byref(nt), C.byref(npt)) == 0
    tags = np.zeros(nt.value + 1, np.uint8)
    pts = np.zeros((npt.value + 1, 2), np.float32)
    assert L.dh_dash(*args, tags.ctypes.data, pts.ctypes.data, nt.value, npt.value, C.byref(nt), C.byref(npt)) == 0
    return tags[: nt.value], pts[: npt.value]


def scenes():
    line = S.single_path_scene([S.MOVE, S.LINE], [[0, 0], [100, 0]], 2.0, join=S.JOIN_ROUND, cap=S.CAP_BUTT)
    line.dashes = [(np.array([10, 5], np.float32), -4.0)]
    sq = S.single_path_scene([S.MOVE, S.LINE, S.LINE, S.LINE, S.CLOSE], [[0, 0], [40, 0], [40, 40], [0, 40]], 1.0,
                             join=S.JOIN_MITER, cap=S.CAP_BUTT)
    sq.dashes = [(np.array([50, 30], np.float32), 20.0)]
    # a dash boundary 2^-20 before a corner at x ~ 1000 (a part without
    # extent), and dashes shorter than the FP32 spacing there
    corner = S.single_path_scene([S.MOVE, S.LINE, S.LINE], [[1000, 0], [1010, 0], [1010, 10]], 2.0,
                                 join=S.JOIN_MITER, cap=S.CAP_BUTT)
    corner.dashes = [(np.array([5, 5], np.float32), 2.0 ** -20)]
    tiny = S.single_path_scene([S.MOVE, S.LINE], [[1000, 0], [1010, 0]], 2.0, join=S.JOIN_MITER, cap=S.CAP_BUTT)
    tiny.dashes = [(np.array([2.0 ** -20, 1.0], np.float32), 0.0)]
    return {
        "line": line,
        "square": sq,
        "ulp_corner": corner,
        "ulp_dashes": tiny,
        # holds dash boundaries within an ulp of segment ends
        "map100k": S.with_dashes(S.scene_c2(2, n_segments=100000, n_paths=1000), seed=4, lo=0.5, hi=12.0),
        "c1": S.with_dashes(S.scene_c1(1), seed=1),
        "c1_fills": S.with_dashes(S.with_fills(S.scene_c1(1), 0.5, seed=3), seed=2),
        "map": S.with_dashes(S.scene_c2(2, n_segments=20000, n_paths=200), seed=4, lo=0.5, hi=12.0),
        "stress": S.with_dashes(S.scene_c3(3, n_cubics=500), seed=6, lo=2.0, hi=30.0),
    }


@pytest.mark.parametrize("name", ["line", "square", "ulp_corner", "ulp_dashes", "c1", "c1_fills", "map", "map100k",
                                  "stress"])
def test_dashing_device_code_matches_the_oracle(lib, name):
    sc = scenes()[name]
    tags, pts = dash_host(lib, sc)
    ref = O.encode_dashed(sc)
    assert ref.status == 0
    assert np.array_equal(tags, ref.tags)
    assert pts.shape == ref.data.shape
    a = pts.view(np.int32).astype(np.int64)
    b = ref.data.view(np.int32).astype(np.int64)
    ulp = np.abs(a - b)
    assert ulp.max() <= 1, (name, int(ulp.max()), int(np.count_nonzero(ulp)))
    assert np.count_nonzero(ulp) <= max(4, 1e-4 * ulp.size)
