"""The C-ABI library loads and exports every entry point declared in include/ndgi.h
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "ndgi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ndgi_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("ndgi_decode", "ndgi_decode_pages", "ndgi_train_step", "ndgi_create",
              "ndgi_bc4_decode_blocks", "ndgi_export", "ndgi_tile_stats"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_2604_12625_amd import ndgi
    if not os.path.exists(ndgi.LIB_PATH):
        pytest.skip("libndgi.so not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(ndgi.LIB_PATH)
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert set(ndgi.EXPORTED) <= set(declared_symbols())


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2604_12625_amd import ndgi
    monkeypatch.setattr(ndgi, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(ndgi, "_lib", None)
    with pytest.raises(ndgi.NdgiError):
        ndgi.lib()
