"""The C-ABI library loads and exports every symbol include/strokex.h
declares (no compute calls: CPU only)."""
import ctypes
import os
import subprocess

import pytest

from paper_2405_00127_amd import binding as B
from paper_2405_00127_amd import build as PB


@pytest.fixture(scope="module")
def built():
    if PB.needs_build():
        PB.build()
    return B.LIB_PATH


def test_header_declares_the_hot_path_calls():
    syms = B.header_symbols()
    for s in ["sx_ctx_create", "sx_scene_encode", "sx_expand", "sx_expand_async", "sx_debug_monoids",
              "sx_debug_counts", "sx_scan_u32", "sx_last_error"]:
        assert s in syms


def test_library_exports_every_declared_symbol(built):
    lib = ctypes.CDLL(built)
    for s in B.header_symbols():
        assert hasattr(lib, s), s
    out = subprocess.run(["nm", "-D", "--defined-only", built], capture_output=True, text=True).stdout
    for s in B.header_symbols():
        assert f" T {s}\n" in out, s


def test_library_is_gfx950_code_object(built):
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", built], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    assert "gfx950" in out.stdout


def test_version_string(built):
    assert b"gfx950" in B.lib().sx_version()


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(RuntimeError):
        B.lib()
