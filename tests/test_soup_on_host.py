"""The single-pass kernel's per-tag body (soup_tag in sx_device.h, the code
the kernel runs) built for the host with the address and undefined-behaviour
sanitizers, on the scene whose first GPU run of that kernel did not finish
(C1) and on arcs, stress cubics and fills: no invalid access, no undefined
behaviour, every record written inside its reservation, the total equal to
the oracle's, and the records the oracle's as multisets.  CPU only."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle as O
from paper_2405_00127_amd import scenes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_00127_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")


class _Paths(C.Structure):
    _fields_ = [("verbs", C.c_void_p), ("verb_off", C.c_void_p), ("pts", C.c_void_p), ("pt_off", C.c_void_p),
                ("style_ix", C.c_void_p), ("xform_ix", C.c_void_p), ("n_paths", C.c_uint32)]


@pytest.fixture(scope="module")
def soup_exe(tmp_path_factory):
    """A host executable is not loadable with sanitizers into this Python, so
    the shim is built as a shared library with the sanitizer runtimes linked
    and run in a child process that preloads them."""
    if not HIPCC:
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("souphost")
    lib = str(d / "libsouphost.so")
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
                           "-ffp-contract=off", "-Wno-unused-command-line-argument",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-sanitize-recover=all",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", lib,
                           os.path.join(os.path.dirname(__file__), "host", "soup_on_host.hip"),
                           os.path.join(CSRC, "sx_encode.cpp")], stderr=subprocess.DEVNULL)
    return lib


_RUNNER = r'''
import ctypes as C, sys, numpy as np
sys.path.insert(0, sys.argv[2]); sys.path.insert(0, sys.argv[3])
from paper_2405_00127_amd import scenes as S
class _Paths(C.Structure):
    _fields_ = [("verbs", C.c_void_p), ("verb_off", C.c_void_p), ("pts", C.c_void_p), ("pt_off", C.c_void_p),
                ("style_ix", C.c_void_p), ("xform_ix", C.c_void_p), ("n_paths", C.c_uint32)]
name = sys.argv[4]
sc = {"c1_lines": lambda: S.scene_c1(1), "c1_arcs": lambda: S.scene_c1(1, output_mode=S.OUT_ARCS),
      "c3_arcs": lambda: S.scene_c3(3, n_cubics=300),
      "c1_fill_shear": lambda: S.with_fills(S.scene_c1(1), 0.5, seed=3, xform=[1.0, 0.2, 0.5, 0.9, 10.0, -5.0])}[name]()
L = C.CDLL(sys.argv[1])
keep = [np.ascontiguousarray(sc.verbs, np.uint8), np.ascontiguousarray(sc.verb_off, np.uint32),
        np.ascontiguousarray(sc.pts, np.float32), np.ascontiguousarray(sc.pt_off, np.uint32),
        np.ascontiguousarray(sc.style_ix, np.uint32), np.ascontiguousarray(sc.xform_ix, np.uint32)]
p = _Paths(*[k.ctypes.data for k in keep], sc.n_paths)
st = np.ascontiguousarray(sc.styles); xf = np.ascontiguousarray(sc.xforms, np.float32)
n, bad = C.c_uint64(), C.c_uint64()
L.soup_expand.argtypes = [C.c_void_p] * 4 + [C.c_uint32, C.c_float, C.c_int, C.c_uint32, C.c_int, C.c_void_p,
                          C.c_uint64, C.c_void_p, C.c_void_p]
w = 6 if sc.output_mode else 5
assert L.soup_expand(C.byref(p), st.ctypes.data, len(st), xf.ctypes.data, len(xf), sc.tolerance, sc.output_mode,
                     16, 0, None, 0, C.byref(n), C.byref(bad)) == 0
cap = n.value
buf = np.zeros(cap * w, np.float32)   # exactly the need: a record past it is an overflow
assert L.soup_expand(C.byref(p), st.ctypes.data, len(st), xf.ctypes.data, len(xf), sc.tolerance, sc.output_mode,
                     16, 0, buf.ctypes.data, cap, C.byref(n), C.byref(bad)) == 0
np.save(sys.argv[5], buf)
print(n.value, bad.value)
'''


def _asan_runtime():
    for name in ("libclang_rt.asan-x86_64.so",):
        out = subprocess.run([HIPCC, "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
        if out and os.path.exists(out):
            return out
        for root in ("/opt/rocm/lib/llvm/lib/clang", "/opt/rocm/llvm/lib/clang"):
            for dirpath, _, files in os.walk(root):
                if name in files:
                    return os.path.join(dirpath, name)
    return None


@pytest.mark.parametrize("name", ["c1_lines", "c1_arcs", "c3_arcs", "c1_fill_shear"])
def test_single_pass_body_under_sanitizers(soup_exe, name, tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("address sanitizer runtime not found")
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = str(tmp_path / "recs.npy")
    r = subprocess.run(["python", "-c", _RUNNER, soup_exe, ROOT, os.path.join(ROOT, "tests"), name, out],
                       capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    n, bad = (int(v) for v in r.stdout.split())
    assert bad == 0
    sc = {"c1_lines": lambda: S.scene_c1(1), "c1_arcs": lambda: S.scene_c1(1, output_mode=S.OUT_ARCS),
          "c3_arcs": lambda: S.scene_c3(3, n_cubics=300),
          "c1_fill_shear": lambda: S.with_fills(S.scene_c1(1), 0.5, seed=3,
                                                xform=[1.0, 0.2, 0.5, 0.9, 10.0, -5.0])}[name]()
    ref = O.expand(sc)
    assert n == len(ref.out)
    w = 6 if sc.output_mode else 5
    recs = np.load(out).reshape(-1, w)
    A = recs[:, :4].astype(np.float64)
    B = np.stack([ref.out["x0"], ref.out["y0"], ref.out["x1"], ref.out["y1"]], 1)
    d1 = cKDTree(B).query(A, p=np.inf)[0]
    d2 = cKDTree(A).query(B, p=np.inf)[0]
    assert max(d1.max(), d2.max()) <= 1e-3
