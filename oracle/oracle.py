"""ctypes wrapper of the plain-C FP64 oracle (``strokex_oracle.c``).

Test infrastructure only: the tests, the smoke check and the benchmark's
CPU-baseline leg call it; the HIP product path never imports it.  The C
source is compiled with gcc into ``liboracle.so`` next to this file.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "strokex_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

FIT_OFFSET, FIT_PAPER = 0, 1
# fit-mode bit: Algorithm 2 without the hodograph test of reading G29
FIT_NO_HODO = 2
# mode bit: exact density integral for line counts, Newton-refined inverse
# for their points (Section 4.2)
DENSITY_NEWTON = 4
KIND_OFFSET, KIND_EVOLUTE, KIND_CONNECT, KIND_JOIN_OUTER, KIND_JOIN_INNER, KIND_CAP = range(6)

OUT_DTYPE = np.dtype(
    [("x0", "<f8"), ("y0", "<f8"), ("x1", "<f8"), ("y1", "<f8"), ("curv", "<f8"),
     ("path", "<u4"), ("kind", "<u4"), ("tag", "<u4")],
    align=True,
)
MARGIN_DTYPE = np.dtype(
    [("fit", "<f8"), ("count", "<f8"), ("rho", "<f8"), ("q", "<f8"), ("len", "<f8"),
     ("join", "<f8"), ("n_pieces", "<u4"), ("max_depth_hits", "<u4")],
    align=True,
)
PIECE_DTYPE = np.dtype(
    [("t0", "<f8"), ("t1", "<f8"), ("k0", "<f8"), ("k1", "<f8"), ("chord", "<f8"),
     ("L", "<f8"), ("th0", "<f8"), ("th1", "<f8"), ("tag", "<u4"), ("forced", "<u4")],
    align=True,
)

# style flag bit 0: the path is filled (flattened at offset 0), not stroked
STYLE_FILL = 1

_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP contraction off, like the paper's math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared", "-o", tmp, SRC, "-lm"]
        )
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = C.CDLL(LIB)
            vp = C.c_void_p
            u32 = C.c_uint32
            L.ox_encode.restype = vp
            L.ox_encode.argtypes = [vp, vp, vp, vp, vp, vp, u32, u32, u32, vp]
            for name, rt in [("ox_enc_status", C.c_int), ("ox_enc_ntags", u32), ("ox_enc_npts", u32),
                             ("ox_enc_nstyles", u32), ("ox_enc_nxforms", u32), ("ox_enc_npaths", u32),
                             ("ox_enc_tags", vp), ("ox_enc_data", vp), ("ox_enc_style_stream", vp),
                             ("ox_enc_xform_stream", vp), ("ox_enc_path_map", vp)]:
                f = getattr(L, name)
                f.restype = rt
                f.argtypes = [vp]
            L.ox_enc_free.argtypes = [vp]
            L.ox_dash_seg_len.restype = C.c_double
            L.ox_dash_seg_len.argtypes = [vp, C.c_int, vp]
            L.ox_encode_dashed.restype = vp
            L.ox_encode_dashed.argtypes = [vp, vp, vp, vp, vp, u32]
            L.ox_monoids.argtypes = [vp, u32, vp, vp, vp, vp]
            L.ox_expand.restype = vp
            L.ox_expand.argtypes = [vp, vp, u32, vp, u32, C.c_double, C.c_int, C.c_int, C.c_int, u32, u32]
            for name, rt in [("ox_res_status", C.c_int), ("ox_res_nout", C.c_uint64), ("ox_res_out", vp),
                             ("ox_res_counts", vp), ("ox_res_margins", vp), ("ox_res_npieces", C.c_uint64),
                             ("ox_res_pieces", vp)]:
                f = getattr(L, name)
                f.restype = rt
                f.argtypes = [vp]
            L.ox_res_free.argtypes = [vp]
            d = C.c_double
            for name, nargs in [("ox_es_k1", 2), ("ox_es_chord", 2), ("ox_f_exact", 1), ("ox_f_approx", 1),
                                ("ox_f_approx_deriv", 1), ("ox_f_approx_inv", 1), ("ox_cubic_area", 4),
                                ("ox_fit_estimate", 4)]:
                f = getattr(L, name)
                f.restype = d
                f.argtypes = [d] * nargs
            L.ox_es_integral.argtypes = [d, d, d, C.POINTER(d), C.POINTER(d)]
            L.ox_line_integral_es.restype = d
            L.ox_line_integral_es.argtypes = [d] * 6 + [C.c_int]
            L.ox_es_side.restype = vp
            L.ox_es_side.argtypes = [d, d, d, d, d, C.c_int, C.c_int]
            L.ox_cubic_chord.argtypes = [vp, d, d, vp]
            L.ox_dens_integral.restype = d
            L.ox_dens_integral.argtypes = [d, d]
            L.ox_f_newton_inv.restype = d
            L.ox_f_newton_inv.argtypes = [d, d, d]
            L.ox_gl_nodes.argtypes = [vp, vp]
            L.ox_xform_ok.restype = C.c_int
            L.ox_xform_ok.argtypes = [vp]
            L.ox_affine_ok.restype = C.c_int
            L.ox_affine_ok.argtypes = [vp]
            assert L.ox_sizeof_out() == OUT_DTYPE.itemsize
            assert L.ox_sizeof_margin() == MARGIN_DTYPE.itemsize
            assert L.ox_sizeof_piece() == PIECE_DTYPE.itemsize
            _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _copy(ptr, dtype, n):
    if n == 0 or not ptr:
        return np.zeros(0, dtype=dtype)
    buf = (C.c_char * (int(n) * np.dtype(dtype).itemsize)).from_address(ptr)
    return np.frombuffer(bytes(buf), dtype=dtype).copy()


# ---------------------------------------------------------------- math pins
def es_k1(th0, th1):
    return lib().ox_es_k1(float(th0), float(th1))


def es_chord(th0, th1):
    return lib().ox_es_chord(float(th0), float(th1))


def f_exact(x):
    return lib().ox_f_exact(float(x))


def f_approx(x):
    return lib().ox_f_approx(float(x))


def f_approx_deriv(x):
    return lib().ox_f_approx_deriv(float(x))


def f_approx_inv(y):
    return lib().ox_f_approx_inv(float(y))


def cubic_area(th0, th1, d0, d1):
    return lib().ox_cubic_area(float(th0), float(th1), float(d0), float(d1))


def fit_estimate(th0, th1, d0, d1):
    return lib().ox_fit_estimate(float(th0), float(th1), float(d0), float(d1))


def es_integral(k0, k1, u):
    re, im = C.c_double(), C.c_double()
    lib().ox_es_integral(float(k0), float(k1), float(u), C.byref(re), C.byref(im))
    return complex(re.value, im.value)


def line_integral_es(k0, k1, L, h, ua, ub, exact=False):
    """Section 4.2 subdivision integral of side h over [ua, ub] of an Euler
    spiral of arc length L (before the sqrt(1/(8 tau_flat)) factor), with
    f_approx or (exact=True) the exact integral."""
    return lib().ox_line_integral_es(float(k0), float(k1), float(L), float(h), float(ua), float(ub), int(bool(exact)))


def cubic_chord(P, t0: float, dt: float) -> np.ndarray:
    """B(t0 + dt) - B(t0) of the cubic P (4 x 2), as the expansion computes
    its sub-cubic chords (test export)."""
    p8 = np.ascontiguousarray(np.asarray(P, np.float64).reshape(8))
    out = np.zeros(2, np.float64)
    lib().ox_cubic_chord(_ptr(p8), float(t0), float(dt), _ptr(out))
    return out


def dens_integral(a, b):
    """int_a^b sqrt|u^2 - 1| du (Section 4.1), integrated directly."""
    return lib().ox_dens_integral(float(a), float(b))


def f_newton_inv(y, lo=-1e300, hi=1e300):
    """x with f(x) = y: the f_approx inverse refined by two Newton steps."""
    return lib().ox_f_newton_inv(float(y), float(lo), float(hi))


def es_side(k0, k1, L, h, tol, mode, flags=0):
    """Records (OUT_DTYPE) of side h of an Euler spiral placed at the origin
    with base angle 0: p(u) = L Z(u), tangent angle phi(u).  flags: 0 or
    DENSITY_NEWTON."""
    L_ = lib()
    hv = C.c_void_p(L_.ox_es_side(float(k0), float(k1), float(L), float(h), float(tol), int(mode), int(flags)))
    if not hv.value:
        raise MemoryError("oracle es_side failed")
    try:
        return _copy(L_.ox_res_out(hv), OUT_DTYPE, L_.ox_res_nout(hv))
    finally:
        L_.ox_res_free(hv)


def gl_nodes():
    x = np.zeros(16)
    w = np.zeros(16)
    lib().ox_gl_nodes(_ptr(x), _ptr(w))
    return x, w


def xform_ok(xf):
    a = np.ascontiguousarray(xf, dtype=np.float32)
    return bool(lib().ox_xform_ok(_ptr(a)))


def affine_ok(xf):
    a = np.ascontiguousarray(xf, dtype=np.float32)
    return bool(lib().ox_affine_ok(_ptr(a)))


# ----------------------------------------------------------------- encoding
@dataclasses.dataclass
class Encoded:
    tags: np.ndarray          # u8 [n_tags]
    data: np.ndarray          # f32 [n_pts, 2]
    style_stream: np.ndarray  # u32: user style index per style entry
    xform_stream: np.ndarray  # u32: user transform index per transform entry
    path_map: np.ndarray      # u32: encoded path -> input path
    status: int
    _h: int = 0

    def __del__(self):
        if self._h:
            lib().ox_enc_free(C.c_void_p(self._h))
            self._h = 0


def encode(scene) -> Encoded:
    L = lib()
    verbs = np.ascontiguousarray(scene.verbs, np.uint8)
    vo = np.ascontiguousarray(scene.verb_off, np.uint32)
    pts = np.ascontiguousarray(scene.pts, np.float32)
    po = np.ascontiguousarray(scene.pt_off, np.uint32)
    si = np.ascontiguousarray(scene.style_ix, np.uint32)
    xi = np.ascontiguousarray(scene.xform_ix, np.uint32)
    # paths drawn as fills (style flag bit 0); an out-of-range style index
    # is left to the encoder, which rejects it
    flags = np.asarray(scene.styles["flags"], np.uint8)
    ok = si < len(flags)
    fill = np.zeros(len(si), np.uint8)
    fill[ok] = flags[si[ok]] & STYLE_FILL
    fill = np.ascontiguousarray(fill)
    h = L.ox_encode(_ptr(verbs), _ptr(vo), _ptr(pts), _ptr(po), _ptr(si), _ptr(xi),
                    scene.n_paths, len(scene.styles), len(scene.xforms), _ptr(fill))
    if not h:
        raise MemoryError("oracle encode failed")
    hv = C.c_void_p(h)
    nt = L.ox_enc_ntags(hv)
    enc = Encoded(
        tags=_copy(L.ox_enc_tags(hv), np.uint8, nt),
        data=_copy(L.ox_enc_data(hv), np.float32, 2 * L.ox_enc_npts(hv)).reshape(-1, 2),
        style_stream=_copy(L.ox_enc_style_stream(hv), np.uint32, L.ox_enc_nstyles(hv)),
        xform_stream=_copy(L.ox_enc_xform_stream(hv), np.uint32, L.ox_enc_nxforms(hv)),
        path_map=_copy(L.ox_enc_path_map(hv), np.uint32, L.ox_enc_npaths(hv)),
        status=L.ox_enc_status(hv),
        _h=h,
    )
    return enc


def dash_seg_len(points) -> float:
    """Arc length of a degree-c Bezier (c + 1 points) by the dashing rule
    (reading G35: 16 panels of 8-node Gauss-Legendre of |B'|)."""
    P = np.ascontiguousarray(np.asarray(points, np.float64).reshape(-1, 2))
    panel = np.zeros(16)
    return lib().ox_dash_seg_len(_ptr(P), len(P) - 1, _ptr(panel))


def encode_dashed(scene, enc: Encoded | None = None) -> Encoded:
    """The dashed encoding of the scene (readings G34-G36): every stroke with
    a dash pattern cut into dashes, each an open subpath."""
    L = lib()
    if enc is None:
        enc = encode(scene)
    vals, off, ph = scene.dash_tables()
    vals = np.ascontiguousarray(vals if len(vals) else np.zeros(1, np.float32))
    fill = np.ascontiguousarray((np.asarray(scene.styles["flags"], np.uint8) & STYLE_FILL).astype(np.uint8))
    h = L.ox_encode_dashed(C.c_void_p(enc._h), _ptr(vals), _ptr(off), _ptr(ph), _ptr(fill), len(scene.styles))
    if not h:
        raise MemoryError("oracle dashed encode failed")
    hv = C.c_void_p(h)
    nt = L.ox_enc_ntags(hv)
    return Encoded(
        tags=_copy(L.ox_enc_tags(hv), np.uint8, nt),
        data=_copy(L.ox_enc_data(hv), np.float32, 2 * L.ox_enc_npts(hv)).reshape(-1, 2),
        style_stream=_copy(L.ox_enc_style_stream(hv), np.uint32, L.ox_enc_nstyles(hv)),
        xform_stream=_copy(L.ox_enc_xform_stream(hv), np.uint32, L.ox_enc_nxforms(hv)),
        path_map=_copy(L.ox_enc_path_map(hv), np.uint32, L.ox_enc_npaths(hv)),
        status=L.ox_enc_status(hv),
        _h=h,
    )


def monoids(tags: np.ndarray) -> np.ndarray:
    """Serial tag-monoid scan; returns u32 [4, n]: data offset, path, style, transform."""
    tags = np.ascontiguousarray(tags, np.uint8)
    n = len(tags)
    out = np.zeros((4, max(n, 1)), dtype=np.uint32)
    lib().ox_monoids(_ptr(tags), n, _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(out[3]))
    return out[:, :n]


# ---------------------------------------------------------------- expansion
@dataclasses.dataclass
class Result:
    status: int
    counts: np.ndarray   # u32 per tag
    out: np.ndarray      # OUT_DTYPE, canonical order
    margins: np.ndarray  # MARGIN_DTYPE per tag
    pieces: np.ndarray   # PIECE_DTYPE
    enc: Encoded

    def offsets(self) -> np.ndarray:
        o = np.zeros(len(self.counts) + 1, dtype=np.uint64)
        o[1:] = np.cumsum(self.counts, dtype=np.uint64)
        return o


def expand_run(scene, tolerance=None, mode=None, tag_begin=0, tag_end=None, enc: Encoded | None = None):
    """Run the full expansion (records emitted) of tags [tag_begin, tag_end)
    and return (status, number of records) without copying anything back:
    the oracle's own work, for timing it."""
    L = lib()
    if enc is None:
        enc = encode(scene)
    tol = scene.tolerance if tolerance is None else tolerance
    mode = scene.output_mode if mode is None else mode
    styles = np.ascontiguousarray(scene.styles)
    xforms = np.ascontiguousarray(scene.xforms, np.float32)
    nt = len(enc.tags)
    h = L.ox_expand(C.c_void_p(enc._h), _ptr(styles), len(styles), _ptr(xforms), len(xforms), float(tol),
                    int(mode), FIT_OFFSET, 1, int(tag_begin), int(nt if tag_end is None else tag_end))
    if not h:
        raise MemoryError("oracle expand failed")
    hv = C.c_void_p(h)
    try:
        return L.ox_res_status(hv), int(L.ox_res_nout(hv))
    finally:
        L.ox_res_free(hv)


def expand(scene, tolerance=None, mode=None, fit_mode=FIT_OFFSET, emit=True,
           tag_begin=0, tag_end=None, enc: Encoded | None = None, margins: bool = True) -> Result:
    """Expand with the oracle (tags [tag_begin, tag_end) of the scene).
    margins=False leaves the per-tag decision margins out of the result
    (they are copied for the whole scene otherwise)."""
    L = lib()
    if enc is None:
        enc = encode(scene)
    if enc.status != 0:
        return Result(enc.status, np.zeros(0, np.uint32), np.zeros(0, OUT_DTYPE),
                      np.zeros(0, MARGIN_DTYPE), np.zeros(0, PIECE_DTYPE), enc)
    tol = scene.tolerance if tolerance is None else tolerance
    mode = scene.output_mode if mode is None else mode
    styles = np.ascontiguousarray(scene.styles)
    xforms = np.ascontiguousarray(scene.xforms, np.float32)
    nt = len(enc.tags)
    if tag_end is None:
        tag_end = nt
    h = L.ox_expand(C.c_void_p(enc._h), _ptr(styles), len(styles), _ptr(xforms), len(xforms),
                    float(tol), int(mode), int(fit_mode), int(bool(emit)), int(tag_begin), int(tag_end))
    if not h:
        raise MemoryError("oracle expand failed")
    hv = C.c_void_p(h)
    try:
        res = Result(
            status=L.ox_res_status(hv),
            counts=_copy(L.ox_res_counts(hv), np.uint32, nt),
            out=_copy(L.ox_res_out(hv), OUT_DTYPE, L.ox_res_nout(hv)),
            margins=_copy(L.ox_res_margins(hv), MARGIN_DTYPE, nt) if margins else np.zeros(0, MARGIN_DTYPE),
            pieces=_copy(L.ox_res_pieces(hv), PIECE_DTYPE, L.ox_res_npieces(hv)),
            enc=enc,
        )
    finally:
        L.ox_res_free(hv)
    return res
