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


def _fake_model(ndgi, W, H, Gw, Gh, T):
    m = ndgi.NdgiModel()
    m.W, m.H, m.Gw, m.Gh, m.T = W, H, Gw, Gh, T
    m.grid_dtype = m.mlp_dtype = ndgi.DTYPE_F16
    m.bc4 = m.grid = m.mlp = 256      # never dereferenced: the size query is host-only
    return m


def test_binned_workspace_size_query():
    """The workspace query is host arithmetic: 512 sort slices x bins of int32 counts,
    bins + 1 int32 starts, bins + 1 int32 work-item offsets, an int32 bin per work item
    (at most n / 2048 + bins items), 4 KiB of column-scan sums, 16 bytes per query, each
    region 256-byte aligned."""
    from paper_2604_12625_amd import ndgi
    if not os.path.exists(ndgi.LIB_PATH):
        pytest.skip("libndgi.so not built (run __graft_entry__.build())")
    L = ndgi.lib()
    b = ctypes.c_int64(-1)
    m = _fake_model(ndgi, 4096, 4096, 1024, 1024, 24)        # 128 x 128 tiles of 32^2
    assert L.ndgi_decode_binned_workspace(ctypes.byref(m), 1 << 24, ctypes.byref(b)) == ndgi.OK
    nb = 128 * 128
    assert b.value == 512 * nb * 4 + 2 * ((nb + 1) * 4 + 252) + 4 * ((1 << 24) // 2048 + nb) + 4096 + 16 * (1 << 24)
    m = _fake_model(ndgi, 8192, 4100, 2048, 1025, 4)          # 64^2 tiles: 128 x 65 bins
    assert L.ndgi_decode_binned_workspace(ctypes.byref(m), 10, ctypes.byref(b)) == ndgi.OK
    nb = 128 * 65
    assert b.value == 512 * nb * 4 + 2 * (((nb + 1) * 4 + 255) // 256 * 256) + (4 * nb + 255) // 256 * 256 + 4096 + 160
    m = _fake_model(ndgi, 16384, 8192, 4096, 2048, 1)         # too many tiles
    assert L.ndgi_decode_binned_workspace(ctypes.byref(m), 10, ctypes.byref(b)) == ndgi.ERR_UNSUPPORTED
    assert b"8192" in L.ndgi_last_error() or b"tiles" in L.ndgi_last_error()
    assert L.ndgi_decode_binned_workspace(ctypes.byref(m), -1, ctypes.byref(b)) == ndgi.ERR_INVALID_ARG
    assert L.ndgi_decode_binned_workspace(ctypes.byref(m), 1 << 31, ctypes.byref(b)) == ndgi.ERR_INVALID_ARG


def test_hybrid_mlp_size_is_host_arithmetic():
    """Packed decoder lengths of the hybrid layout: 16-h-h-3 with biases."""
    from paper_2604_12625_amd import ndgi
    if not os.path.exists(ndgi.LIB_PATH):
        pytest.skip("libndgi.so not built (run __graft_entry__.build())")
    assert ndgi.hybrid_mlp_size(16) == 16 * 16 + 16 + 16 * 16 + 16 + 3 * 16 + 3 == 595
    assert ndgi.hybrid_mlp_size(64) == 64 * 16 + 64 + 64 * 64 + 64 + 3 * 64 + 3 == 5443
    assert ndgi.hybrid_mlp_size(32) == -1


def test_product_package_never_imports_the_oracle():
    """The oracle is test infrastructure: no source of the package names it, and importing
    every module of the package leaves it out of sys.modules."""
    import importlib
    import subprocess
    import sys
    pkg = os.path.join(ROOT, "paper_2604_12625_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b", src), os.path.join(dirpath, f)
    mods = [f[:-3] for f in os.listdir(pkg) if f.endswith(".py") and f != "__init__.py"]
    code = ("import sys; sys.path.insert(0, %r)\n" % ROOT +
            "".join(f"import paper_2604_12625_amd.{m}\n" for m in sorted(mods)) +
            "bad = [m for m in sys.modules if m == 'oracle' or m.startswith('oracle.')]\n"
            "assert not bad, bad\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr


def test_npz_checkpoint_format_round_trips_without_pickle(tmp_path):
    """Checkpoints and saved models are plain .npz arrays: numbers, strings and arrays come
    back as they went in, through a loader that refuses pickled objects."""
    import numpy as np
    from paper_2604_12625_amd import ndgi as N
    d = dict(kind="ndgi_train", W=64, lr=1e-3, step=7, a=np.arange(6, dtype=np.float32).reshape(2, 3),
             keys=np.zeros(0, np.float32))
    p = tmp_path / "c.npz"
    np.savez(p, **N.to_npz(d))
    with np.load(p, allow_pickle=False) as z:
        assert set(z.files) == set(d)
    back = N.from_npz(p)
    assert back["kind"] == "ndgi_train" and back["W"] == 64 and back["step"] == 7
    assert isinstance(back["W"], int) and abs(back["lr"] - 1e-3) < 1e-18
    np.testing.assert_array_equal(back["a"], d["a"])
    assert back["keys"].shape == (0,)
