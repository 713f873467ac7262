"""Thin Python binding of libndgi.so (ctypes).

Argument marshalling only: every step of the decode and training path runs in the HIP
kernels behind the C ABI (include/ndgi.h).  PyTorch provides device memory and the
current stream.  Loading fails loudly when the library has not been built; there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libndgi.so")

OK, ERR_INVALID_ARG, ERR_UNSUPPORTED, ERR_HIP, ERR_OOM = 0, -1, -2, -3, -4
DTYPE_F32, DTYPE_F16 = 0, 1
PREC_F32, PREC_F16 = 0, 1
FLAG_BAD_PAGE_REQUEST = 1
FLAG_BAD_SAMPLE = 2
MLP_SIZE = 1699
TRAIN_FORWARD, TRAIN_BACKWARD, TRAIN_LOSS_GRAD, TRAIN_FUSED, TRAIN_ADAM, TRAIN_ZERO_GRAD = range(6)

EXPORTED = (
    "ndgi_create", "ndgi_destroy", "ndgi_last_error", "ndgi_get_error_flags",
    "ndgi_bc4_decode_blocks", "ndgi_bc7_decode_blocks", "ndgi_decode", "ndgi_decode_pages", "ndgi_decode_pages_graph",
    "ndgi_set_launch", "ndgi_train_param_count", "ndgi_train_step", "ndgi_export",
    "ndgi_tile_stats", "ndgi_decode_binned_workspace", "ndgi_decode_binned", "ndgi_decode_binned_noalloc", "ndgi_reserve_decode",
    "ndgi_hybrid_mlp_size", "ndgi_hybrid_decode", "ndgi_hybrid_decode_pages",
    "ndgi_hybrid_decode_pages_graph", "ndgi_hybrid_train_param_count", "ndgi_hybrid_train_step",
    "ndgi_hybrid_export", "ndgi_hybrid_normalize_target", "ndgi_hybrid_restore",
)
HTRAIN_BCSIM, HTRAIN_NOISE, HTRAIN_QPLANES, HTRAIN_DIRECT = 1, 2, 4, 8
CODEC_BC4, CODEC_BC7 = 0, 1


class NdgiModel(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("Gw", C.c_int32), ("Gh", C.c_int32),
                ("T", C.c_int32), ("grid_dtype", C.c_int32), ("mlp_dtype", C.c_int32),
                ("reserved0", C.c_int32), ("bc4", C.c_void_p), ("grid", C.c_void_p),
                ("mlp", C.c_void_p), ("reserved1", C.c_void_p)]


class NdgiPageReq(C.Structure):
    _fields_ = [("model", C.c_int32), ("page_x", C.c_int32), ("page_y", C.c_int32),
                ("t", C.c_float), ("dst_offset", C.c_int64)]


class NdgiTrainState(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("Gw", C.c_int32), ("Gh", C.c_int32),
                ("T", C.c_int32), ("reserved0", C.c_int32), ("params", C.c_void_p),
                ("grads", C.c_void_p), ("adam_m", C.c_void_p), ("adam_v", C.c_void_p),
                ("step", C.c_int64), ("lr_feat", C.c_float), ("lr_mlp", C.c_float),
                ("beta1", C.c_float), ("beta2", C.c_float), ("eps", C.c_float),
                ("reserved1", C.c_float)]


class NdgiBatch(C.Structure):
    _fields_ = [("samples", C.c_void_p), ("n", C.c_int64), ("target", C.c_void_p),
                ("pred", C.c_void_p), ("grad_pred", C.c_void_p)]


class NdgiHybridModel(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("Gu", C.c_int32), ("Gv", C.c_int32),
                ("S", C.c_int32), ("U", C.c_int32), ("V", C.c_int32), ("Tt", C.c_int32),
                ("hidden", C.c_int32), ("mlp_dtype", C.c_int32), ("n_keys", C.c_int32),
                ("codec", C.c_int32), ("fuv", C.c_void_p), ("fuvt", C.c_void_p),
                ("fut", C.c_void_p), ("fvt", C.c_void_p), ("keys", C.c_void_p), ("mlp", C.c_void_p)]


class NdgiHybridTrainState(C.Structure):
    _fields_ = [("W", C.c_int32), ("H", C.c_int32), ("Gu", C.c_int32), ("Gv", C.c_int32),
                ("S", C.c_int32), ("U", C.c_int32), ("V", C.c_int32), ("Tt", C.c_int32),
                ("hidden", C.c_int32), ("frames", C.c_int32), ("n_models", C.c_int32),
                ("per_model", C.c_int32), ("codec", C.c_int32), ("reserved0", C.c_int32),
                ("keys", C.c_void_p),
                ("params", C.c_void_p), ("grads", C.c_void_p), ("adam_m", C.c_void_p),
                ("adam_v", C.c_void_p), ("step", C.c_int64), ("lr_feat", C.c_float),
                ("lr_mlp", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("seed", C.c_uint32)]


class NdgiHybridBatch(C.Structure):
    _fields_ = [("samples", C.c_void_p), ("n", C.c_int64), ("target", C.c_void_p), ("pred", C.c_void_p)]


assert C.sizeof(NdgiModel) == 64 and C.sizeof(NdgiPageReq) == 24 and C.sizeof(NdgiHybridModel) == 96
assert C.sizeof(NdgiHybridTrainState) == 128 and C.sizeof(NdgiHybridBatch) == 32


class NdgiError(RuntimeError):
    pass


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NdgiError(f"{LIB_PATH} not found: build it with "
                            "`python -m paper_2604_12625_amd.build` (no CPU fallback exists)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.ndgi_create.argtypes = [C.POINTER(vp), i32]
        L.ndgi_destroy.argtypes = [vp]
        L.ndgi_last_error.restype = C.c_char_p
        L.ndgi_get_error_flags.argtypes = [vp, vp, C.POINTER(C.c_uint32)]
        L.ndgi_bc4_decode_blocks.argtypes = [vp, i64, vp, vp]
        L.ndgi_bc7_decode_blocks.argtypes = [vp, i64, vp, vp]
        L.ndgi_bc4_decode_blocks_impl.argtypes = [vp, i64, vp, i32, vp]
        L.ndgi_bc4_encode_blocks.argtypes = [vp, i64, vp, vp]
        L.ndgi_bc7_encode_blocks.argtypes = [vp, i64, vp, vp]
        L.ndgi_decode.argtypes = [vp, C.POINTER(NdgiModel), vp, i64, vp, i32, vp]
        pages = [vp, vp, i32, vp, vp, i32, i32, vp, i64, i32, vp]
        L.ndgi_decode_pages.argtypes = pages
        L.ndgi_decode_pages_graph.argtypes = pages
        L.ndgi_set_launch.argtypes = [vp, i32, i32, i32]
        L.ndgi_train_param_count.argtypes = [i32, i32, i32, i32, i32]
        L.ndgi_train_param_count.restype = i64
        L.ndgi_train_step.argtypes = [vp, C.POINTER(NdgiTrainState), C.POINTER(NdgiBatch), i32, vp, vp]
        L.ndgi_export.argtypes = [vp, C.POINTER(NdgiTrainState), vp, vp, i32, vp, i32, vp]
        L.ndgi_tile_stats.argtypes = [vp, vp, i32, vp, i32, i32, i32, vp, vp]
        L.ndgi_psnr.argtypes = [vp, vp, i32, i32, i32, i32, vp, vp, vp]
        L.ndgi_decode_binned_workspace.argtypes = [C.POINTER(NdgiModel), i64, C.POINTER(i64)]
        L.ndgi_decode_binned.argtypes = [vp, C.POINTER(NdgiModel), vp, i64, vp, i32, vp, i64, vp]
        L.ndgi_decode_binned_noalloc.argtypes = [vp, C.POINTER(NdgiModel), vp, i64, vp, i32, vp]
        L.ndgi_reserve_decode.argtypes = [vp, C.POINTER(NdgiModel), i64]
        L.ndgi_hybrid_mlp_size.argtypes = [i32]
        L.ndgi_hybrid_mlp_size.restype = i32
        L.ndgi_hybrid_decode.argtypes = [vp, C.POINTER(NdgiHybridModel), vp, i64, vp, i32, vp]
        hpages = [vp, vp, i32, vp, vp, i32, i32, vp, i64, i32, i32, i32, vp]
        L.ndgi_hybrid_decode_pages.argtypes = hpages
        L.ndgi_hybrid_decode_pages_graph.argtypes = hpages
        L.ndgi_hybrid_train_param_count.argtypes = [i32] * 10
        L.ndgi_hybrid_train_param_count.restype = i64
        L.ndgi_hybrid_train_step.argtypes = [vp, C.POINTER(NdgiHybridTrainState), C.POINTER(NdgiHybridBatch), i32,
                                             i32, vp, vp]
        L.ndgi_hybrid_export.argtypes = [vp, C.POINTER(NdgiHybridTrainState), i32, vp, vp, vp, vp, vp, i32, vp]
        L.ndgi_hybrid_encode.argtypes = [vp, C.POINTER(NdgiHybridTrainState), i32, i32, i32, vp, vp, vp, vp, vp, i32,
                                         vp]
        L.ndgi_hybrid_import.argtypes = [vp, C.POINTER(NdgiHybridModel), C.POINTER(NdgiHybridTrainState), i32, vp]
        L.ndgi_hybrid_normalize_target.argtypes = [vp, vp, i32, i32, i32, C.c_float, vp, vp, vp]
        L.ndgi_hybrid_restore.argtypes = [vp, vp, i32, i64, vp, C.c_float, vp, vp]
        _lib = L
    return _lib


def check(rc: int, what: str = ""):
    if rc != OK:
        msg = lib().ndgi_last_error().decode(errors="replace")
        raise NdgiError(f"{what} failed ({rc}): {msg}")


def _ptr(t) -> int:
    return 0 if t is None else t.data_ptr()


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class DeviceModel:
    """A compressed model whose arrays live in device memory (torch tensors)."""

    def __init__(self, W, H, Gw, Gh, T, bc4, grid, mlp):
        import torch
        self.W, self.H, self.Gw, self.Gh, self.T = int(W), int(H), int(Gw), int(Gh), int(T)
        self.bc4 = bc4.contiguous()
        self.grid = grid.contiguous()
        self.mlp = mlp.contiguous()
        dt = {torch.float32: DTYPE_F32, torch.float16: DTYPE_F16}
        self.desc = NdgiModel(self.W, self.H, self.Gw, self.Gh, self.T, dt[self.grid.dtype],
                              dt[self.mlp.dtype], 0, self.bc4.data_ptr(), self.grid.data_ptr(),
                              self.mlp.data_ptr(), None)

    @classmethod
    def from_numpy(cls, m: dict, device="cuda"):
        import torch
        return cls(m["W"], m["H"], m["Gw"], m["Gh"], m["T"],
                   torch.from_numpy(m["bc4"]).to(device),
                   torch.from_numpy(m["grid"]).to(device),
                   torch.from_numpy(m["mlp"]).to(device))

    def desc_bytes(self) -> bytes:
        return bytes(self.desc)

    def to_numpy(self) -> dict:
        """Host copy in from_numpy's layout."""
        return dict(W=self.W, H=self.H, Gw=self.Gw, Gh=self.Gh, T=self.T, bc4=self.bc4.cpu().numpy(),
                    grid=self.grid.cpu().numpy(), mlp=self.mlp.cpu().numpy())

    def save(self, path):
        """The compressed model as an .npz file (arrays only, no pickled objects)."""
        np.savez(path, **to_npz(self.to_numpy()))

    @classmethod
    def load(cls, path, device="cuda"):
        return cls.from_numpy(from_npz(path), device)


class HybridModel:
    """A model in the paper's hybrid layout (F_uv, F_uvt, F_ut, F_vt, key times, decoder)
    whose arrays live in device memory (torch tensors)."""

    def __init__(self, W, H, Gu, Gv, S, U, V, Tt, hidden, fuv, fuvt, fut, fvt, keys, mlp, codec=CODEC_BC4):
        import torch
        self.arrays = [a.contiguous() for a in (fuv, fuvt, fut, fvt, keys, mlp)]
        fuv, fuvt, fut, fvt, keys, mlp = self.arrays
        dt = {torch.float32: DTYPE_F32, torch.float16: DTYPE_F16}
        nk = keys.numel()
        self.desc = NdgiHybridModel(int(W), int(H), int(Gu), int(Gv), int(S), int(U), int(V), int(Tt),
                                    int(hidden), dt[mlp.dtype], nk, int(codec), fuv.data_ptr(), fuvt.data_ptr(),
                                    fut.data_ptr(), fvt.data_ptr(), keys.data_ptr() if nk else None,
                                    mlp.data_ptr())

    @classmethod
    def from_numpy(cls, m: dict, device="cuda"):
        import torch
        t = {k: torch.from_numpy(m[k]).to(device) for k in ("fuv", "fuvt", "fut", "fvt", "keys", "mlp")}
        return cls(m["W"], m["H"], m["Gu"], m["Gv"], m["S"], m["U"], m["V"], m["Tt"], m["hidden"],
                   t["fuv"], t["fuvt"], t["fut"], t["fvt"], t["keys"].to(torch.float32), t["mlp"],
                   m.get("codec", CODEC_BC4))

    def desc_bytes(self) -> bytes:
        return bytes(self.desc)

    def to_numpy(self) -> dict:
        """Host copy in from_numpy's layout."""
        d = self.desc
        out = dict(W=d.W, H=d.H, Gu=d.Gu, Gv=d.Gv, S=d.S, U=d.U, V=d.V, Tt=d.Tt, hidden=d.hidden, codec=d.codec)
        for k, a in zip(("fuv", "fuvt", "fut", "fvt", "keys", "mlp"), self.arrays):
            out[k] = a.cpu().numpy()
        return out

    def save(self, path):
        """The compressed model as an .npz file (arrays only, no pickled objects)."""
        np.savez(path, **to_npz(self.to_numpy()))

    @classmethod
    def load(cls, path, device="cuda"):
        return cls.from_numpy(from_npz(path), device)


def to_npz(d: dict) -> dict:
    """A dict of numbers, strings and arrays as .npz entries: each value becomes an array."""
    return {k: np.asarray(v) for k, v in d.items()}


def from_npz(path) -> dict:
    """Inverse of to_npz (allow_pickle stays off): 0-d arrays become Python scalars."""
    with np.load(path) as z:
        return {k: (z[k].item() if z[k].ndim == 0 else z[k]) for k in z.files}


def hybrid_mlp_size(hidden: int) -> int:
    return int(lib().ndgi_hybrid_mlp_size(hidden))


class Context:
    """Owns an ndgi_ctx on one device."""

    def __init__(self, device: int = 0):
        self.h = C.c_void_p()
        check(lib().ndgi_create(C.byref(self.h), device), "ndgi_create")

    def close(self):
        if self.h:
            h, self.h = self.h, C.c_void_p()
            check(lib().ndgi_destroy(h), "ndgi_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ decode
    def decode(self, model: DeviceModel, uvt, prec=PREC_F16, out=None, stream=None):
        import torch
        n = uvt.shape[0]
        if out is None:
            out = torch.empty((n, 3), dtype=torch.float16 if prec == PREC_F16 else torch.float32,
                              device=uvt.device)
        check(lib().ndgi_decode(self.h, C.byref(model.desc), _ptr(uvt), n, _ptr(out), prec,
                                _stream(stream)), "ndgi_decode")
        return out

    def binned_workspace_bytes(self, model: DeviceModel, n: int) -> int:
        b = C.c_int64(0)
        check(lib().ndgi_decode_binned_workspace(C.byref(model.desc), n, C.byref(b)),
              "ndgi_decode_binned_workspace")
        return b.value

    def decode_binned(self, model: DeviceModel, uvt, prec=PREC_F16, out=None, workspace=None,
                      stream=None):
        """Binned decode; `workspace` is a uint8 device tensor reused across calls
        (allocated here when None or too small, returned with the output)."""
        import torch
        n = uvt.shape[0]
        if out is None:
            out = torch.empty((n, 3), dtype=torch.float16 if prec == PREC_F16 else torch.float32,
                              device=uvt.device)
        need = self.binned_workspace_bytes(model, n)
        if workspace is None or workspace.numel() < need:
            workspace = torch.empty(max(need, 256), dtype=torch.uint8, device=uvt.device)
        check(lib().ndgi_decode_binned(self.h, C.byref(model.desc), _ptr(uvt), n, _ptr(out), prec,
                                       _ptr(workspace), workspace.numel(), _stream(stream)),
              "ndgi_decode_binned")
        return out, workspace

    def reserve_decode(self, model, max_queries: int):
        """Reserve the context's decode workspace (ndgi_reserve_decode): later decode() calls
        with many queries per tile run the binned kernels; max_queries = 0 releases it."""
        check(lib().ndgi_reserve_decode(self.h, C.byref(model.desc) if model is not None else None, max_queries),
              "ndgi_reserve_decode")

    def decode_binned_noalloc(self, model: DeviceModel, uvt, out, prec=PREC_F16, stream=None):
        """Binned decode into the caller's `out` through the library's static scratch
        (allocates nothing, takes no workspace)."""
        check(lib().ndgi_decode_binned_noalloc(self.h, C.byref(model.desc), _ptr(uvt), uvt.shape[0], _ptr(out),
                                               prec, _stream(stream)), "ndgi_decode_binned_noalloc")
        return out

    def decode_pages(self, models_dev, n_models, reqs_dev, n_reqs_dev, max_reqs, page, dst,
                     pitch, prec=PREC_F16, graph=False, stream=None):
        f = lib().ndgi_decode_pages_graph if graph else lib().ndgi_decode_pages
        check(f(self.h, _ptr(models_dev), n_models, _ptr(reqs_dev), _ptr(n_reqs_dev), max_reqs,
                page, _ptr(dst), pitch, prec, _stream(stream)), "ndgi_decode_pages")
        return dst

    def hybrid_decode(self, model: HybridModel, uvt, prec=PREC_F16, out=None, stream=None):
        import torch
        n = uvt.shape[0]
        if out is None:
            out = torch.empty((n, 3), dtype=torch.float16 if prec == PREC_F16 else torch.float32,
                              device=uvt.device)
        check(lib().ndgi_hybrid_decode(self.h, C.byref(model.desc), _ptr(uvt), n, _ptr(out), prec,
                                       _stream(stream)), "ndgi_hybrid_decode")
        return out

    def hybrid_decode_pages(self, models_dev, n_models, reqs_dev, n_reqs_dev, max_reqs, page, dst,
                            pitch, prec=PREC_F16, widths=0, border=0, graph=False, stream=None):
        """widths: bit 0 = models of hidden width 16 present, bit 1 = width 64; 0 = either.
        border: texels of mirrored border around each page (regions of (page + 2 border)^2)."""
        f = lib().ndgi_hybrid_decode_pages_graph if graph else lib().ndgi_hybrid_decode_pages
        check(f(self.h, _ptr(models_dev), n_models, _ptr(reqs_dev), _ptr(n_reqs_dev), max_reqs,
                page, _ptr(dst), pitch, prec, widths, border, _stream(stream)), "ndgi_hybrid_decode_pages")
        return dst

    def set_launch(self, tile_w, tile_h, waves_per_cu):
        check(lib().ndgi_set_launch(self.h, tile_w, tile_h, waves_per_cu), "ndgi_set_launch")

    def tile_stats(self, pred, target_bits, W, H, tile=128, out=None, stream=None):
        """Per-tile (max target, min target, squared error) in FP64 for one [H][W][3] map."""
        import torch
        ny, nx = (H + tile - 1) // tile, (W + tile - 1) // tile
        if out is None:
            out = torch.empty((ny, nx, 3), dtype=torch.float64, device=pred.device)
        pdt = DTYPE_F16 if pred.dtype == torch.float16 else DTYPE_F32
        check(lib().ndgi_tile_stats(self.h, _ptr(pred), pdt, _ptr(target_bits), W, H, tile, _ptr(out),
                                    _stream(stream)), "ndgi_tile_stats")
        return out

    def psnr(self, stats, W, H, tile=128, stream=None) -> dict:
        """Tiled PSNR (ndgi_psnr) of stacked per-map tile statistics [n][ny][nx][3] (device
        FP64): dict(tiled, global, min, p10, scored, tiles, tile_db) with the per-tile dB on the
        device (NaN for skipped tiles)."""
        import torch
        stats = stats.contiguous()
        n = stats.shape[0] if stats.dim() == 4 else 1
        tile_db = torch.empty(stats.shape[:-1], dtype=torch.float64, device=stats.device)
        summ = torch.empty(5, dtype=torch.float64, device=stats.device)
        check(lib().ndgi_psnr(self.h, _ptr(stats), n, W, H, tile, _ptr(tile_db), _ptr(summ), _stream(stream)),
              "ndgi_psnr")
        v = summ.cpu().tolist()
        scored = tile_db[~torch.isnan(tile_db)]
        p10 = float(torch.quantile(scored, 0.1).item()) if scored.numel() else float("nan")
        return dict(tiled=v[0], **{"global": v[1]}, min=v[2], p10=p10, scored=int(v[3]), tiles=int(v[4]),
                    tile_db=tile_db)

    def error_flags(self, stream=None) -> int:
        f = C.c_uint32(0)
        check(lib().ndgi_get_error_flags(self.h, _stream(stream), C.byref(f)), "ndgi_get_error_flags")
        return f.value


def bc4_decode_blocks(blocks, out=None, stream=None, impl=None):
    """Decode [n][8] uint8 device blocks to [n][16] uint8 (impl: one of the kernels' texel
    decoders, ndgi_bc4_decode_blocks_impl)."""
    import torch
    n = blocks.shape[0]
    if out is None:
        out = torch.empty((n, 16), dtype=torch.uint8, device=blocks.device)
    if impl is None:
        check(lib().ndgi_bc4_decode_blocks(_ptr(blocks), n, _ptr(out), _stream(stream)), "ndgi_bc4_decode_blocks")
    else:
        check(lib().ndgi_bc4_decode_blocks_impl(_ptr(blocks), n, _ptr(out), int(impl), _stream(stream)),
              "ndgi_bc4_decode_blocks_impl")
    return out


def bc7_decode_blocks(blocks, out=None, stream=None):
    """Decode [n][16] uint8 device BC7 blocks (modes 4, 5 and 6; other modes decode to 0) to
    [n][16 texels][4 channels] uint8."""
    import torch
    n = blocks.shape[0]
    if out is None:
        out = torch.empty((n, 16, 4), dtype=torch.uint8, device=blocks.device)
    check(lib().ndgi_bc7_decode_blocks(_ptr(blocks), n, _ptr(out), _stream(stream)), "ndgi_bc7_decode_blocks")
    return out


def bc4_encode_blocks(texels, out=None, stream=None):
    """Encode [n][16] uint8 device texels as [n][8] BC4 blocks (the exhaustive optimum)."""
    import torch
    n = texels.shape[0]
    if out is None:
        out = torch.empty((n, 8), dtype=torch.uint8, device=texels.device)
    check(lib().ndgi_bc4_encode_blocks(_ptr(texels), n, _ptr(out), _stream(stream)), "ndgi_bc4_encode_blocks")
    return out


def bc7_encode_blocks(texels, out=None, stream=None):
    """Encode [n][16][4] uint8 device texels as [n][16] BC7 blocks (modes 6, 5 and 4, each
    block its least-error candidate)."""
    import torch
    n = texels.shape[0]
    if out is None:
        out = torch.empty((n, 16), dtype=torch.uint8, device=texels.device)
    check(lib().ndgi_bc7_encode_blocks(_ptr(texels), n, _ptr(out), _stream(stream)), "ndgi_bc7_encode_blocks")
    return out


def models_array(models, device="cuda"):
    """Device array of ndgi_model (or ndgi_hybrid_model) descriptors (keeps no reference to
    the models)."""
    import torch
    raw = b"".join(m.desc_bytes() for m in models)
    return torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)


def page_requests(model, px, py, t, dst_offset, device="cuda"):
    """Device array of ndgi_page_req from equal-length sequences."""
    import numpy as np
    import torch
    n = len(model)
    rec = np.zeros(n, dtype=np.dtype([("model", "<i4"), ("px", "<i4"), ("py", "<i4"),
                                       ("t", "<f4"), ("off", "<i8")]))
    rec["model"], rec["px"], rec["py"], rec["t"], rec["off"] = model, px, py, t, dst_offset
    return torch.from_numpy(rec.view(np.uint8).copy()).to(device)
