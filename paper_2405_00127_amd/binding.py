"""Thin ctypes binding of libstrokex.so (include/strokex.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  PyTorch supplies device memory (tensors) and streams.  Loading
fails loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re
import threading
from typing import Optional

import numpy as np

from . import scenes as S

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libstrokex.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "strokex.h")

SX_OK, SX_EINVAL, SX_ENOMEM, SX_EDEVICE, SX_ETOOSMALL, SX_EBUSY = 0, -1, -2, -3, -4, -5
OUT_LINES, OUT_ARCS = 0, 1
(PHASE_SCAN_TAGS, PHASE_BISECT_COUNT, PHASE_SCAN_SLOTS, PHASE_BISECT_WRITE, PHASE_PIECES, PHASE_TAILS,
 PHASE_SCAN_RECORDS, PHASE_RECORDS) = range(8)
PHASE_NAMES = ["scan_tags", "bisect_count", "scan_slots", "bisect_write", "pieces", "tails", "scan_records",
               "records"]
RECORD_BYTES = {OUT_LINES: 20, OUT_ARCS: 24}

LINE_DTYPE = np.dtype([("x0", "<f4"), ("y0", "<f4"), ("x1", "<f4"), ("y1", "<f4"), ("path", "<u4")])
ARC_DTYPE = np.dtype([("x0", "<f4"), ("y0", "<f4"), ("x1", "<f4"), ("y1", "<f4"), ("curv", "<f4"), ("path", "<u4")])


class StrokexError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"strokex error {code}: {msg}")
        self.code = code


class _Paths(C.Structure):
    _fields_ = [("verbs", C.c_void_p), ("verb_off", C.c_void_p), ("pts", C.c_void_p), ("pt_off", C.c_void_p),
                ("style_ix", C.c_void_p), ("xform_ix", C.c_void_p), ("n_paths", C.c_uint32)]


class _Config(C.Structure):
    _fields_ = [("fit_mode", C.c_uint32), ("density", C.c_uint32), ("constants_version", C.c_uint32),
                ("reserved", C.c_uint32)]


FIT_OFFSET, FIT_PAPER = 0, 1
DENSITY_APPROX, DENSITY_NEWTON = 0, 1
CONSTANTS_VERSION = 1


class _Dash(C.Structure):
    _fields_ = [("array", C.c_void_p), ("count", C.c_uint32), ("offset", C.c_float)]


class _Tuning(C.Structure):
    _fields_ = [("piece_waves", C.c_uint32), ("chunk_k", C.c_uint32), ("bisect_range", C.c_uint32),
                ("bisect_waves", C.c_uint32)]


_lib = None
_lock = threading.Lock()


def header_symbols():
    """Function names declared in include/strokex.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(sx_\w+)\s*\(", txt, re.M)))


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
            L = C.CDLL(LIB_PATH)
            vp, u32, u64 = C.c_void_p, C.c_uint32, C.c_uint64
            sig = {
                "sx_ctx_create": (C.c_int, [C.c_int, C.POINTER(_Config), C.POINTER(vp)]),
                "sx_get_config": (C.c_int, [vp, C.POINTER(_Config)]),
                "sx_ctx_destroy": (C.c_int, [vp]),
                "sx_last_error": (C.c_char_p, [vp]),
                "sx_version": (C.c_char_p, []),
                "sx_scene_encode": (C.c_int, [vp, C.POINTER(_Paths), vp, u32, vp, u32, vp, C.POINTER(vp)]),
                "sx_scene_release": (C.c_int, [vp, vp]),
                "sx_scene_encode_dashed": (C.c_int, [vp, C.POINTER(_Paths), vp, vp, u32, vp, u32, vp,
                                                     C.POINTER(vp)]),
                "sx_scene_dash_ms": (C.c_int, [vp, C.POINTER(C.c_float)]),
                "sx_scene_info": (C.c_int, [vp, vp, vp, vp, vp, vp]),
                "sx_scene_download": (C.c_int, [vp, vp, vp, vp]),
                "sx_expand": (C.c_int, [vp, vp, C.c_float, C.c_int, vp, u64, C.POINTER(u64), vp]),
                "sx_expand_async": (C.c_int, [vp, vp, C.c_float, C.c_int, vp, u64, vp, vp]),
                "sx_debug_monoids": (C.c_int, [vp, vp, vp, vp]),
                "sx_debug_counts": (C.c_int, [vp, vp, C.c_float, C.c_int, vp, vp]),
                "sx_debug_offsets": (C.c_int, [vp, vp, C.c_float, C.c_int, vp, vp]),
                "sx_scan_u32": (C.c_int, [vp, vp, vp, u32, vp]),
                "sx_scan_u32_noalloc": (C.c_int, [vp, vp, vp, u32, vp]),
                "sx_run_phase": (C.c_int, [vp, vp, C.c_int, C.c_float, C.c_int, vp, u64, vp]),
                "sx_set_tuning": (C.c_int, [vp, C.POINTER(_Tuning)]),
                "sx_batch_create": (C.c_int, [vp, C.POINTER(vp)]),
                "sx_debug_piece_stats": (C.c_int, [vp, vp, C.c_float, C.c_int, vp, vp]),
                "sx_batch_destroy": (C.c_int, [vp, vp]),
                "sx_batch_set": (C.c_int, [vp, vp, vp, u32, vp]),
                "sx_batch_info": (C.c_int, [vp, vp, C.POINTER(vp)]),
                "sx_batch_expand": (C.c_int, [vp, vp, C.c_float, C.c_int, vp, u64, vp, vp, vp]),
                "sx_get_tuning": (C.c_int, [vp, C.POINTER(_Tuning)]),
                "sx_expand_soup": (C.c_int, [vp, vp, C.c_float, C.c_int, vp, u64, C.POINTER(u64), vp]),
                "sx_scene_estimate": (C.c_int, [vp, C.c_float, C.c_int, C.POINTER(u64)]),
            }
            for name, (res, args) in sig.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
    return _lib


def _arr(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _stream_ptr(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Scene:
    """A device-resident encoded scene (owned by its Context)."""

    def __init__(self, ctx: "Context", handle: int, src: S.Scene):
        self.ctx = ctx
        self.h = handle
        self.src = src
        nt, npt, np_, ns, nx = (C.c_uint32() for _ in range(5))
        lib().sx_scene_info(C.c_void_p(handle), C.byref(nt), C.byref(npt), C.byref(np_), C.byref(ns), C.byref(nx))
        self.n_tags, self.n_pts, self.n_paths = nt.value, npt.value, np_.value
        self.n_styles, self.n_xforms = ns.value, nx.value

    def dash_ms(self) -> float:
        """Device milliseconds of the dashing passes (0 for an undashed scene)."""
        v = C.c_float()
        lib().sx_scene_dash_ms(C.c_void_p(self.h), C.byref(v))
        return float(v.value)

    def release(self):
        if self.h:
            lib().sx_scene_release(C.c_void_p(self.ctx.h), C.c_void_p(self.h))
            self.h = 0

    def __del__(self):
        try:
            if self.h and self.ctx.h:
                self.release()
        except Exception:
            pass

    def download(self):
        tags = np.zeros(self.n_tags, np.uint8)
        data = np.zeros((self.n_pts, 2), np.float32)
        pm = np.zeros(self.n_paths, np.uint32)
        rc = lib().sx_scene_download(C.c_void_p(self.h), tags.ctypes.data, data.ctypes.data, pm.ctypes.data)
        if rc:
            raise StrokexError(rc, "download")
        return tags, data, pm


class Context:
    """A library context on one device.  fit_mode: FIT_OFFSET (default) or
    FIT_PAPER; density: DENSITY_APPROX (default) or DENSITY_NEWTON (see
    sx_config in include/strokex.h)."""

    def __init__(self, device: int = 0, fit_mode: int = FIT_OFFSET, density: int = DENSITY_APPROX):
        self.h = 0
        h = C.c_void_p()
        cfg = _Config(int(fit_mode), int(density), CONSTANTS_VERSION, 0)
        rc = lib().sx_ctx_create(int(device), C.byref(cfg), C.byref(h))
        if rc != SX_OK:
            raise StrokexError(rc, "sx_ctx_create failed (bad configuration, or no gfx950 GPU visible?)")
        self.h = h.value
        self.device = device

    def config(self) -> dict:
        c = _Config()
        self._check(lib().sx_get_config(C.c_void_p(self.h), C.byref(c)), "sx_get_config")
        return {"fit_mode": c.fit_mode, "density": c.density, "constants_version": c.constants_version}

    def close(self):
        if self.h:
            lib().sx_ctx_destroy(C.c_void_p(self.h))
            self.h = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != SX_OK:
            msg = lib().sx_last_error(C.c_void_p(self.h)).decode()
            raise StrokexError(rc, f"{what}: {msg}")

    def encode(self, scene: S.Scene, stream=None) -> Scene:
        keep = dict(
            verbs=_arr(scene.verbs, np.uint8), verb_off=_arr(scene.verb_off, np.uint32),
            pts=_arr(scene.pts, np.float32), pt_off=_arr(scene.pt_off, np.uint32),
            style_ix=_arr(scene.style_ix, np.uint32), xform_ix=_arr(scene.xform_ix, np.uint32),
            styles=_arr(scene.styles, S.STYLE_DTYPE), xforms=_arr(scene.xforms, np.float32),
        )
        p = _Paths(keep["verbs"].ctypes.data, keep["verb_off"].ctypes.data, keep["pts"].ctypes.data,
                   keep["pt_off"].ctypes.data, keep["style_ix"].ctypes.data, keep["xform_ix"].ctypes.data,
                   scene.n_paths)
        out = C.c_void_p()
        if scene.dashes is not None:
            # per style: its pattern (None: solid)
            n = len(keep["styles"])
            arrs = [np.ascontiguousarray((scene.dashes[k][0] if k < len(scene.dashes) and scene.dashes[k] is not None
                                          else np.zeros(0)), np.float32) for k in range(n)]
            tab = (_Dash * max(1, n))()
            for k in range(n):
                d = scene.dashes[k] if k < len(scene.dashes) else None
                tab[k] = _Dash(arrs[k].ctypes.data if len(arrs[k]) else None, len(arrs[k]),
                               float(d[1]) if d is not None else 0.0)
            rc = lib().sx_scene_encode_dashed(C.c_void_p(self.h), C.byref(p), keep["styles"].ctypes.data, tab, n,
                                              keep["xforms"].ctypes.data, len(keep["xforms"]), _stream_ptr(stream),
                                              C.byref(out))
            self._check(rc, "sx_scene_encode_dashed")
        else:
            rc = lib().sx_scene_encode(C.c_void_p(self.h), C.byref(p), keep["styles"].ctypes.data,
                                       len(keep["styles"]), keep["xforms"].ctypes.data, len(keep["xforms"]),
                                       _stream_ptr(stream), C.byref(out))
            self._check(rc, "sx_scene_encode")
        return Scene(self, out.value, scene)

    def expand_into(self, scene: Scene, out_ptr: int, capacity_bytes: int, tolerance: float, mode: int,
                    stream=None) -> int:
        """Raw call: returns the record count; raises on SX_ETOOSMALL."""
        cnt = C.c_uint64()
        rc = lib().sx_expand(C.c_void_p(self.h), C.c_void_p(scene.h), float(tolerance), int(mode),
                             C.c_void_p(out_ptr), int(capacity_bytes), C.byref(cnt), _stream_ptr(stream))
        if rc == SX_ETOOSMALL:
            e = StrokexError(rc, "output buffer too small")
            e.required = cnt.value
            raise e
        self._check(rc, "sx_expand")
        return cnt.value

    def expand_soup_into(self, scene: Scene, out_ptr: int, capacity_bytes: int, tolerance: float, mode: int,
                         stream=None) -> int:
        """Single-pass expansion (unordered line soup); returns the record count,
        raises on SX_ETOOSMALL with .required set."""
        cnt = C.c_uint64()
        rc = lib().sx_expand_soup(C.c_void_p(self.h), C.c_void_p(scene.h), float(tolerance), int(mode),
                                  C.c_void_p(out_ptr), int(capacity_bytes), C.byref(cnt), _stream_ptr(stream))
        if rc == SX_ETOOSMALL:
            e = StrokexError(rc, "output buffer too small")
            e.required = cnt.value
            raise e
        self._check(rc, "sx_expand_soup")
        return cnt.value

    def estimate(self, scene: Scene, tolerance: Optional[float] = None, mode: Optional[int] = None) -> int:
        """Host-side estimate of the records the scene needs (Wang's formula)."""
        tol = scene.src.tolerance if tolerance is None else tolerance
        mode = scene.src.output_mode if mode is None else mode
        n = C.c_uint64()
        self._check(lib().sx_scene_estimate(C.c_void_p(scene.h), float(tol), int(mode), C.byref(n)),
                    "sx_scene_estimate")
        return n.value

    def expand_soup(self, scene: Scene, tolerance: Optional[float] = None, mode: Optional[int] = None,
                    stream=None):
        """Single-pass expansion into a buffer sized by the estimate; a short
        buffer is regrown to the reported need and the call repeated once.
        Returns (records view [n, 5|6] float32, count, buffer, retried)."""
        import torch

        tol = scene.src.tolerance if tolerance is None else tolerance
        mode = scene.src.output_mode if mode is None else mode
        rec = RECORD_BYTES[mode]
        cap = max(1, self.estimate(scene, tol, mode))
        out = torch.empty(cap * rec, dtype=torch.uint8, device=f"cuda:{self.device}")
        retried = False
        try:
            n = self.expand_soup_into(scene, out.data_ptr(), out.numel(), tol, mode, stream)
        except StrokexError as e:
            if e.code != SX_ETOOSMALL:
                raise
            retried = True
            out = torch.empty(max(1, e.required) * rec, dtype=torch.uint8, device=out.device)
            n = self.expand_soup_into(scene, out.data_ptr(), out.numel(), tol, mode, stream)
        return out[: n * rec].view(torch.float32).view(-1, rec // 4), n, out, retried

    def expand_async(self, scene: Scene, out_ptr: int, capacity_bytes: int, count_dev_ptr: int, tolerance: float,
                     mode: int, stream=None):
        """count_dev_ptr: two device uint64 (records; 0 or the item workspace needed)."""
        rc = lib().sx_expand_async(C.c_void_p(self.h), C.c_void_p(scene.h), float(tolerance), int(mode),
                                   C.c_void_p(out_ptr), int(capacity_bytes), C.c_void_p(count_dev_ptr),
                                   _stream_ptr(stream))
        self._check(rc, "sx_expand_async")

    def expand(self, scene: Scene, tolerance: Optional[float] = None, mode: Optional[int] = None, out=None,
               stream=None):
        """Expand into a torch uint8 device tensor (grown on demand).
        Returns (records tensor view [n, 5|6] float32 (path id bits in the last
        column), count, buffer)."""
        import torch

        tol = scene.src.tolerance if tolerance is None else tolerance
        mode = scene.src.output_mode if mode is None else mode
        rec = RECORD_BYTES[mode]
        if out is None:
            out = torch.empty(max(1, scene.n_tags * 16) * rec, dtype=torch.uint8, device=f"cuda:{self.device}")
        while True:
            try:
                n = self.expand_into(scene, out.data_ptr(), out.numel(), tol, mode, stream)
                break
            except StrokexError as e:
                if e.code != SX_ETOOSMALL:
                    raise
                out = torch.empty(int(e.required * 1.25 + 1) * rec, dtype=torch.uint8, device=out.device)
        return out[: n * rec].view(torch.float32).view(-1, rec // 4), n, out

    def set_tuning(self, piece_waves: int = None, chunk_k: int = None, bisect_range: int = None,
                   bisect_waves: int = None):
        """Set launch parameters (unspecified ones keep their value)."""
        cur = self.get_tuning() if self.h else {}
        t = _Tuning(int(piece_waves if piece_waves is not None else cur["piece_waves"]),
                    int(chunk_k if chunk_k is not None else cur["chunk_k"]),
                    int(bisect_range if bisect_range is not None else cur["bisect_range"]),
                    int(bisect_waves if bisect_waves is not None else cur["bisect_waves"]))
        self._check(lib().sx_set_tuning(C.c_void_p(self.h), C.byref(t)), "sx_set_tuning")

    def get_tuning(self):
        t = _Tuning()
        self._check(lib().sx_get_tuning(C.c_void_p(self.h), C.byref(t)), "sx_get_tuning")
        return {"piece_waves": t.piece_waves, "chunk_k": t.chunk_k, "bisect_range": t.bisect_range,
                "bisect_waves": t.bisect_waves}

    def piece_stats(self, scene: Scene, tolerance=None, mode=None, stream=None) -> dict:
        """Work counts of the piece phase (instrumented run; synchronous)."""
        tol = scene.src.tolerance if tolerance is None else tolerance
        mode = scene.src.output_mode if mode is None else mode
        st = (C.c_uint64 * 6)()
        self._check(lib().sx_debug_piece_stats(C.c_void_p(self.h), C.c_void_p(scene.h), float(tol), int(mode), st,
                                               _stream_ptr(stream)), "sx_debug_piece_stats")
        keys = ["trials", "pieces", "ranges", "evolutes", "joins", "lines"]
        return {k: int(v) for k, v in zip(keys, st)}

    def run_phase(self, scene: Scene, phase: int, tolerance: float, mode: int, out_ptr: int = 0,
                  capacity_bytes: int = 0, stream=None):
        rc = lib().sx_run_phase(C.c_void_p(self.h), C.c_void_p(scene.h), int(phase), float(tolerance), int(mode),
                                C.c_void_p(out_ptr), int(capacity_bytes), _stream_ptr(stream))
        self._check(rc, "sx_run_phase")

    def monoids(self, scene: Scene, stream=None):
        import torch

        m = torch.empty(4 * max(scene.n_tags, 1), dtype=torch.int32, device=f"cuda:{self.device}")
        self._check(lib().sx_debug_monoids(C.c_void_p(self.h), C.c_void_p(scene.h), C.c_void_p(m.data_ptr()),
                                           _stream_ptr(stream)), "sx_debug_monoids")
        return m[: 4 * scene.n_tags].view(4, -1)

    def counts(self, scene: Scene, tolerance=None, mode=None, stream=None):
        import torch

        tol = scene.src.tolerance if tolerance is None else tolerance
        mode = scene.src.output_mode if mode is None else mode
        c = torch.empty(max(scene.n_tags, 1), dtype=torch.int32, device=f"cuda:{self.device}")
        self._check(lib().sx_debug_counts(C.c_void_p(self.h), C.c_void_p(scene.h), float(tol), int(mode),
                                          C.c_void_p(c.data_ptr()), _stream_ptr(stream)), "sx_debug_counts")
        return c[: scene.n_tags]

    def offsets(self, scene: Scene, tolerance=None, mode=None, stream=None):
        import torch

        tol = scene.src.tolerance if tolerance is None else tolerance
        mode = scene.src.output_mode if mode is None else mode
        o = torch.empty(scene.n_tags + 1, dtype=torch.int64, device=f"cuda:{self.device}")
        self._check(lib().sx_debug_offsets(C.c_void_p(self.h), C.c_void_p(scene.h), float(tol), int(mode),
                                           C.c_void_p(o.data_ptr()), _stream_ptr(stream)), "sx_debug_offsets")
        return o

    def scan_u32(self, values, stream=None):
        import torch

        n = int(values.numel())
        out = torch.empty(n + 1, dtype=torch.int64, device=values.device)
        self._check(lib().sx_scan_u32(C.c_void_p(self.h), C.c_void_p(values.data_ptr()), C.c_void_p(out.data_ptr()),
                                      n, _stream_ptr(stream)), "sx_scan_u32")
        return out


    def scan_u32_noalloc(self, values, out=None, stream=None):
        """sx_scan_u32_noalloc into `out` (int64, n + 1; allocated here when
        None -- the library call itself allocates nothing)."""
        import torch

        n = int(values.numel())
        if out is None:
            out = torch.empty(n + 1, dtype=torch.int64, device=values.device)
        self._check(lib().sx_scan_u32_noalloc(C.c_void_p(self.h), C.c_void_p(values.data_ptr()),
                                              C.c_void_p(out.data_ptr()), n, _stream_ptr(stream)),
                    "sx_scan_u32_noalloc")
        return out


class Batch:
    """Many encoded scenes concatenated in one device arena and expanded by
    one pipeline (``sx_batch_*``).  Keeps the member scenes alive."""

    def __init__(self, ctx: "Context"):
        self.ctx = ctx
        h = C.c_void_p()
        ctx._check(lib().sx_batch_create(C.c_void_p(ctx.h), C.byref(h)), "sx_batch_create")
        self.h = h.value
        self.scenes = []

    def set(self, scenes, stream=None):
        arr = (C.c_void_p * max(1, len(scenes)))(*[sc.h for sc in scenes])
        self.ctx._check(lib().sx_batch_set(C.c_void_p(self.ctx.h), C.c_void_p(self.h), arr, len(scenes),
                                           _stream_ptr(stream)), "sx_batch_set")
        self.scenes = list(scenes)

    @property
    def n_scenes(self) -> int:
        return len(self.scenes)

    def arena(self) -> "Scene":
        """The arena as a scene handle (owned by the batch: never released)."""
        a = C.c_void_p()
        n = C.c_uint32()
        self.ctx._check(lib().sx_batch_info(C.c_void_p(self.h), C.byref(n), C.byref(a)), "sx_batch_info")
        return _ArenaScene(self.ctx, a.value)

    def expand_async(self, tolerance: float, mode: int, out_ptr: int, capacity_bytes: int, scene_offsets_ptr: int,
                     status_ptr: int, stream=None):
        rc = lib().sx_batch_expand(C.c_void_p(self.ctx.h), C.c_void_p(self.h), float(tolerance), int(mode),
                                   C.c_void_p(out_ptr), int(capacity_bytes), C.c_void_p(scene_offsets_ptr),
                                   C.c_void_p(status_ptr), _stream_ptr(stream))
        self.ctx._check(rc, "sx_batch_expand")

    def prepare(self, tolerance: float, mode: int, stream=None, headroom: float = 1.0):
        """Size the output and the arena's item workspace with one synchronous
        expansion; returns (output uint8 tensor, scene offsets tensor (n+1),
        status tensor (2)), all device int64 / uint8 torch tensors."""
        import torch

        dev = f"cuda:{self.ctx.device}"
        arena = self.arena()
        rec = RECORD_BYTES[mode]
        probe = torch.empty(16, dtype=torch.uint8, device=dev)
        try:
            n = self.ctx.expand_into(arena, probe.data_ptr(), 0, tolerance, mode, stream)
        except StrokexError as e:
            if e.code != SX_ETOOSMALL:
                raise
            n = e.required
        out = torch.empty(max(1, int(n * headroom)) * rec, dtype=torch.uint8, device=dev)
        offs = torch.zeros(self.n_scenes + 1, dtype=torch.int64, device=dev)
        status = torch.zeros(2, dtype=torch.int64, device=dev)
        return out, offs, status

    def destroy(self):
        if self.h:
            lib().sx_batch_destroy(C.c_void_p(self.ctx.h), C.c_void_p(self.h))
            self.h = None
            self.scenes = []

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class _ArenaScene:
    """Scene-shaped view of a batch arena (for sx_expand sizing)."""

    def __init__(self, ctx, h):
        self.ctx = ctx
        self.h = h
        n = C.c_uint32()
        lib().sx_scene_info(C.c_void_p(h), C.byref(n), None, None, None, None)
        self.n_tags = n.value


def records_to_numpy(recs_tensor, mode) -> np.ndarray:
    a = recs_tensor.detach().cpu().numpy()
    return np.ascontiguousarray(a).view(LINE_DTYPE if mode == OUT_LINES else ARC_DTYPE).reshape(-1)
