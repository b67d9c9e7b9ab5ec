"""The library's host path encoder (Section 8.2, Table 1), compiled for the
host with g++ through a small shim, against the oracle's encoder: tags, the
point stream, the style / transform streams and the path map, bit-exact, on
seeded scenes with strokes, fills (every subpath closed), closepaths,
degenerate segments and style / transform changes.  CPU only."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_2405_00127_amd import scenes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_00127_amd", "csrc")


class _Paths(C.Structure):
    _fields_ = [("verbs", C.c_void_p), ("verb_off", C.c_void_p), ("pts", C.c_void_p), ("pt_off", C.c_void_p),
                ("style_ix", C.c_void_p), ("xform_ix", C.c_void_p), ("n_paths", C.c_uint32)]


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("shim") / "libencshim.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", os.path.join(ROOT, "include"),
                           "-I", CSRC, "-o", out, os.path.join(os.path.dirname(__file__), "host", "encode_shim.cpp"),
                           os.path.join(CSRC, "sx_encode.cpp")])
    L = C.CDLL(out)
    L.shim_encode.argtypes = [C.POINTER(_Paths), C.c_void_p, C.c_uint32, C.c_uint32]
    L.shim_error.restype = C.c_char_p
    for n in ("shim_n_tags", "shim_n_data", "shim_n_styles", "shim_n_xforms", "shim_n_paths"):
        getattr(L, n).restype = C.c_uint32
    L.shim_copy.argtypes = [C.c_void_p] * 5
    return L


def _encode(L, sc):
    keep = [np.ascontiguousarray(sc.verbs, np.uint8), np.ascontiguousarray(sc.verb_off, np.uint32),
            np.ascontiguousarray(sc.pts, np.float32), np.ascontiguousarray(sc.pt_off, np.uint32),
            np.ascontiguousarray(sc.style_ix, np.uint32), np.ascontiguousarray(sc.xform_ix, np.uint32)]
    p = _Paths(*[k.ctypes.data for k in keep], sc.n_paths)
    st = np.ascontiguousarray(sc.styles)
    rc = L.shim_encode(C.byref(p), st.ctypes.data, len(st), len(sc.xforms))
    if rc != 0:
        return rc, None
    tags = np.zeros(L.shim_n_tags(), np.uint8)
    data = np.zeros(L.shim_n_data(), np.float32)
    ss = np.zeros(L.shim_n_styles(), np.uint32)
    xs = np.zeros(L.shim_n_xforms(), np.uint32)
    pm = np.zeros(L.shim_n_paths(), np.uint32)
    L.shim_copy(tags.ctypes.data, data.ctypes.data, ss.ctypes.data, xs.ctypes.data, pm.ctypes.data)
    return 0, (tags, data.reshape(-1, 2), ss, xs, pm)


def _degenerate_scene():
    b = S.SceneBuilder()
    b.add_path([0], [[1, 1]], 0, 0)                                      # moveto only
    b.add_path([0, 1, 1], [[2, 2], [2, 2], [2, 2]], 1, 0)                # zero-length segments
    b.add_path([0, 1, 4, 1, 1], [[0, 0], [5, 0], [9, 9], [3, 4]], 1, 0)  # closepath then more segments
    b.add_path([0, 3, 0, 2], [[0, 0], [0, 0], [5, 5], [9, 0], [1, 1], [2, 3], [4, 1]], 0, 0)
    b.add_path([0, 1, 1, 1], [[0, 0], [10, 0], [10, 10], [0, 0]], 1, 0)  # ends at its start
    st = S.make_styles([1.0, 2.0], S.JOIN_ROUND, S.CAP_BUTT)
    st["flags"][1] = S.STYLE_FILL
    return b.build(st, S.identity_xforms())


@pytest.mark.parametrize("name", ["c1", "c1_fills", "c2_mixed", "c3", "degenerate"])
def test_host_encoder_matches_the_oracle(shim, name):
    sc = {"c1": lambda: S.scene_c1(1),
          "c1_fills": lambda: S.with_fills(S.scene_c1(1), 0.5, seed=3, xform=[1.0, 0.2, 0.5, 0.9, 10.0, -5.0]),
          "c2_mixed": lambda: S.with_fills(S.scene_c2(2, n_segments=30000, n_paths=300), 0.4, seed=7),
          "c3": lambda: S.scene_c3(3, n_cubics=500),
          "degenerate": _degenerate_scene}[name]()
    rc, got = _encode(shim, sc)
    e = O.encode(sc)
    assert rc == 0 and e.status == 0
    tags, data, ss, xs, pm = got
    assert np.array_equal(tags, e.tags)
    assert np.array_equal(data.view(np.uint32), e.data.view(np.uint32))
    assert np.array_equal(ss, e.style_stream) and np.array_equal(xs, e.xform_stream)
    assert np.array_equal(pm, e.path_map)


@pytest.mark.parametrize("bad", ["no_move", "nan", "style_ix", "count"])
def test_host_encoder_rejects_what_the_oracle_rejects(shim, bad):
    verbs, pts, six = [0, 1], [[0, 0], [1, 0]], 0
    if bad == "no_move":
        verbs, pts = [1], [[1, 0]]
    elif bad == "nan":
        pts = [[0, 0], [np.nan, 0]]
    elif bad == "style_ix":
        six = 5
    b = S.SceneBuilder()
    b.add_path(verbs, pts, six, 0)
    sc = b.build(S.make_styles([1.0], S.JOIN_ROUND, S.CAP_BUTT), S.identity_xforms())
    if bad == "count":
        sc.pt_off = sc.pt_off.copy()
        sc.pt_off[-1] += 1
        sc.pts = np.concatenate([sc.pts, [[7.0, 7.0]]]).astype(np.float32)
    rc, _ = _encode(shim, sc)
    assert rc == -1
    assert O.encode(sc).status == -1
