"""Fit of the paper's hybrid layout to a temporal lightmap with its training recipe (Sec. 3.4,
Sec. 4), all on the GPU kernels, then export, decode and score.

Target: a 128 x 128 tile (the paper trains one model per VT tile) cut from the synthetic
1024^2 temporal lightmap, baked at 26 key times (24 hourly plus two around a light switch,
like the paper's sets), FP16.  Preprocessing: gamma 2.2 and per-frame, per-channel mean
normalisation.  Training: Adam at the paper's learning rate 1e-3 and batch 2^12 texel
samples; phase 1 with BC simulation of F_uv / F_uvt and noise on the sampled features;
phase 2 fine-tunes the decoder on frozen features as a decode sees them.  Export (BC7
mode-6 blocks as in the paper, or BC4 blocks per channel; 8-bit planes, FP16 decoder), decode of all 26 frames through the page decoder at
their key times (FP16 and FP32 paths), inverse preprocessing, tiled PSNR (one 128^2 tile
per frame).  The same run without the BC simulation in phase 1 is the simulation's
ablation (Table 7 of the paper, on synthetic data).
"""
from __future__ import annotations

import sys
import time

import numpy as np

TILE = 128
GAMMA = 2.2
BATCH = 1 << 12
LR = 1e-3


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def tile_target(torch, I, keys, x0=384, y0=512, scene_side=1024, seed=6):
    """[frames][TILE][TILE][3] FP16 target: a tile of the synthetic scene at the key times."""
    scene = I.light_scene(scene_side, scene_side, I.rng(seed, I.P_TARGET))
    frames = []
    for t in keys:
        f = I.scene_frame_torch(scene, float(t), device="cuda", rows=(y0, y0 + TILE))
        frames.append(f[:, x0:x0 + TILE].to(torch.float16))
    return torch.stack(frames).contiguous()


def fit(torch, N, I, ctx, init, target_bits, steps1, steps2, bcsim: bool, seed=0):
    from .train import HybridTrainer, hybrid_normalize_target
    frames = target_bits.shape[0]
    tgt, means = hybrid_normalize_target(ctx, target_bits.view(torch.int16), GAMMA)
    tr = HybridTrainer(ctx, init, lr_feat=LR, lr_mlp=LR, seed=seed)
    smp = torch.stack([I.train_samples_torch(BATCH, TILE, TILE, frames, seed=70_000 + i)
                       for i in range(steps1 + steps2)])
    f1 = (N.HTRAIN_BCSIM if bcsim else 0) | N.HTRAIN_NOISE
    f2 = N.HTRAIN_BCSIM | N.HTRAIN_QPLANES
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(steps1):
        tr.step(smp[i], tgt, f1)
        if (i + 1) % 1000 == 0:
            losses.append((i + 1, float(tr.loss.item())))
    e1.record()
    e1.synchronize()
    ms1 = e0.elapsed_time(e1)
    tr.set_lr(lr_feat=0.0)
    for i in range(steps1, steps1 + steps2):
        tr.step(smp[i], tgt, f2)
    torch.cuda.synchronize()
    losses.append((steps1 + steps2, float(tr.loss.item())))
    wall = time.perf_counter() - t0
    return tr, means, dict(train_ms_per_step=ms1 / steps1, wall_s=wall, loss_curve=losses, flags_phase1=f1,
                           flags_phase2=f2, n_params=int(tr.n_params))


def score(torch, N, ctx, tr, means, target_bits, keys):
    """Tiled PSNR of the exported model's decode (FP16 and FP32 paths) against the target."""
    from .train import hybrid_restore
    frames = target_bits.shape[0]
    hm = tr.export(N.DTYPE_F16)
    marr = N.models_array([hm])
    rq = N.page_requests(np.zeros(frames, np.int32), np.zeros(frames, np.int32), np.zeros(frames, np.int32),
                         np.asarray(keys, np.float32), (np.arange(frames) * TILE * TILE).astype(np.int64))
    nreq = torch.tensor([frames], dtype=torch.int32, device="cuda")
    width = 2 if tr.d["hidden"] == 64 else 1
    out = {}
    for prec, name in ((N.PREC_F16, "f16"), (N.PREC_F32, "f32")):
        dst = torch.empty((frames * TILE * TILE, 3), dtype=torch.float16 if prec == N.PREC_F16 else torch.float32,
                          device="cuda")
        ctx.hybrid_decode_pages(marr, 1, rq, nreq, frames, TILE, dst, TILE, prec, widths=width)
        stats = []
        for f in range(frames):
            rec = hybrid_restore(ctx, dst[f * TILE * TILE:(f + 1) * TILE * TILE], means[f], GAMMA)
            stats.append(ctx.tile_stats(rec, target_bits[f].view(torch.int16), TILE, TILE, TILE).cpu().numpy())
        tiled, glob = N.psnr_from_stats(stats, TILE, TILE, TILE)
        out[name] = dict(psnr_tiled_db=tiled, psnr_global_db=glob)
    assert ctx.error_flags() == 0
    return out


def _codec(args):
    return 0 if getattr(args, "codec", "bc7") == "bc4" else 1


def _bits(codec):
    return 8 if codec == 1 else 16     # F_uv / F_uvt bits per texel: one BC7 block or four BC4 blocks


def run_hfit(args, torch, N, I, ctx, profile="M", steps1=4000, steps2=1000):
    keys = I.lightmap_key_times(I.rng(6, I.P_MODEL, 1))
    target = tile_target(torch, I, keys)
    codec = _codec(args)
    init = I.hybrid_train_init(TILE, TILE, profile, len(keys), keys, I.rng(6, I.P_INIT), codec=codec)
    side, hidden = I.HYBRID_PROFILES[profile]
    runs = {}
    for name, bc in (("recipe", True), ("without_bc_simulation", False)):
        tr, means, info = fit(torch, N, I, ctx, init, target, steps1, steps2, bc)
        info["decode"] = score(torch, N, ctx, tr, means, target, keys)
        runs[name] = info
        _log(f"hybrid fit {profile} {name}: {info['train_ms_per_step']:.3f} ms/step, loss {info['loss_curve'][-1][1]:.4e}, "
             f"PSNR FP16 {info['decode']['f16']['psnr_tiled_db']:.2f} dB, FP32 {info['decode']['f32']['psnr_tiled_db']:.2f} dB")
    return {
        "metric": "hybrid-layout fit: tiled PSNR after export, train ms/step",
        "config": {"workload": f"one {TILE}x{TILE} tile of the synthetic 1024^2 temporal lightmap at 26 key times; "
                               f"profile {profile} (F_uvt {side}^2 x 12 x 4, hidden {hidden}); "
                               f"{'BC7 mode 6' if codec else 'BC4'} F_uv / F_uvt; batch {BATCH}, Adam "
                               f"lr {LR}; {steps1} steps with BC simulation and noise, {steps2} decoder fine-tune "
                               "steps on frozen features; gamma 2.2 + per-frame mean normalisation"},
        "data": "synthetic", "codec": "bc7" if codec else "bc4",
        "train_params": int(runs["recipe"].get("n_params", 0)) or None,
        "bits_per_texel": bits_per_texel_hybrid(TILE, TILE, len(keys), side, 12, (64, 64, 24), hidden, _bits(codec)),
        "runs": runs,
    }


def bits_per_texel_hybrid(W, H, frames, side, slices, plane, hidden, uv_bits_per_texel):
    """Stored bits per texel per frame of a hybrid model: F_uv and the F_uvt slices at
    `uv_bits_per_texel` (16 for four BC4 channels, 8 for the paper's BC7), 8-bit planes,
    FP16 decoder."""
    U, V, Tt = plane
    mlp = hidden * 16 + hidden + hidden * hidden + hidden + 3 * hidden + 3
    bits = W * H * uv_bits_per_texel + side * side * slices * uv_bits_per_texel + (U + V) * Tt * 2 * 8 + mlp * 16
    return bits / (W * H * frames)


def run_hfit_map(args, torch, N, I, ctx, profile="M", side=1024, steps1=6000, steps2=2000):
    """The paper's production setting: a side x side lightmap as (side/128)^2 per-tile models,
    trained together in one launch per step (4096 samples per model), exported, and decoded
    for all 26 frames through the page decoder (one request per tile and frame, one launch).
    Tiles carry a mirrored border of `--border` texels (Sec. 6; 4 by default): training
    samples are drawn over the mirror-padded tile and each decoded page is a
    (128 + 2 border)^2 region; PSNR is scored on the 128^2 interiors."""
    from .train import HybridTrainer, hybrid_normalize_target, hybrid_restore
    keys = I.lightmap_key_times(I.rng(6, I.P_MODEL, 1))
    frames = len(keys)
    nt = side // TILE
    M = nt * nt
    scene = I.light_scene(side, side, I.rng(7, I.P_TARGET))
    full = torch.stack([I.scene_frame_torch(scene, float(t), device="cuda").to(torch.float16) for t in keys])
    # tile-major target [M][frames][TILE][TILE][3]
    tiles = full.view(frames, nt, TILE, nt, TILE, 3).permute(1, 3, 0, 2, 4, 5).reshape(M, frames, TILE, TILE, 3)
    tiles = tiles.contiguous()
    tgt, means = hybrid_normalize_target(ctx, tiles.view(M * frames, TILE, TILE, 3).view(torch.int16), GAMMA)
    codec = _codec(args)
    border = int(getattr(args, "border", 4))
    R = TILE + 2 * border                       # stored page side
    inits = [I.hybrid_train_init(TILE, TILE, profile, frames, keys, I.rng(7, I.P_INIT, m), codec=codec)
             for m in range(M)]
    tr = HybridTrainer(ctx, inits, lr_feat=LR, lr_mlp=LR, seed=1, per_model=BATCH)
    _log(f"hybrid map: {M} tile models, {tr.n_params / 1e6:.2f} M parameters")
    n_steps = steps1 + steps2
    f1, f2 = N.HTRAIN_BCSIM | N.HTRAIN_NOISE, N.HTRAIN_BCSIM | N.HTRAIN_QPLANES
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    losses = []
    torch.cuda.synchronize()
    e0.record()
    for i in range(n_steps):
        if i == steps1:
            tr.set_lr(lr_feat=0.0)
        smp = I.train_samples_torch(M * BATCH, TILE, TILE, frames, seed=90_000 + i, border=border)
        tr.step(smp, tgt, f1 if i < steps1 else f2)
        if (i + 1) % 1000 == 0:
            losses.append((i + 1, float(tr.loss.item())))
    e1.record()
    e1.synchronize()
    train_ms = e0.elapsed_time(e1)
    # export every tile model and decode all frames in one page launch
    models = [tr.export(N.DTYPE_F16, model=m) for m in range(M)]
    marr = N.models_array(models)
    mi = np.repeat(np.arange(M), frames).astype(np.int32)
    fi = np.tile(np.arange(frames), M)
    rq = N.page_requests(mi, np.zeros(M * frames, np.int32), np.zeros(M * frames, np.int32),
                         np.asarray(keys, np.float32)[fi], (np.arange(M * frames) * R * R).astype(np.int64))
    nreq = torch.tensor([M * frames], dtype=torch.int32, device="cuda")
    width = 2 if I.HYBRID_PROFILES[profile][1] == 64 else 1
    out = {}
    for prec, name in ((N.PREC_F16, "f16"), (N.PREC_F32, "f32")):
        dst = torch.empty((M * frames * R * R, 3), dtype=torch.float16 if prec == N.PREC_F16 else torch.float32,
                          device="cuda")
        ctx.hybrid_decode_pages(marr, M, rq, nreq, M * frames, TILE, dst, R, prec, widths=width, border=border)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record()
        ctx.hybrid_decode_pages(marr, M, rq, nreq, M * frames, TILE, dst, R, prec, widths=width, border=border)
        ev1.record()
        ev1.synchronize()
        inner = dst.view(M * frames, R, R, 3)[:, border:border + TILE, border:border + TILE].contiguous()
        inner = inner.view(M * frames * TILE * TILE, 3)
        stats = []
        for k in range(M * frames):
            rec = hybrid_restore(ctx, inner[k * TILE * TILE:(k + 1) * TILE * TILE], means[k], GAMMA)
            stats.append(ctx.tile_stats(rec, tiles.view(M * frames, TILE, TILE, 3)[k].view(torch.int16), TILE, TILE,
                                        TILE).cpu().numpy())
        tiled, glob = N.psnr_from_stats(stats, TILE, TILE, TILE)
        out[name] = dict(psnr_tiled_db=tiled, psnr_global_db=glob, decode_all_frames_ms=ev0.elapsed_time(ev1))
        _log(f"hybrid map {name}: PSNR tiled {tiled:.2f} dB, decode of {frames} frames "
             f"({R}^2 pages) {out[name]['decode_all_frames_ms']:.3f} ms")
    assert ctx.error_flags() == 0
    s_uvt, hidden = I.HYBRID_PROFILES[profile]
    return {
        "metric": "hybrid-layout map fit: per-tile models trained together, tiled PSNR after export",
        "config": {"workload": f"{side}x{side} synthetic temporal lightmap at 26 key times as {M} tile models of "
                               f"{TILE}^2 with {border}-texel mirrored borders, profile {profile}, "
                               f"{'BC7 mode 6' if codec else 'BC4'} F_uv / F_uvt; "
                               f"batch {BATCH} per model, Adam lr {LR}; {steps1} steps with "
                               f"BC simulation and noise, {steps2} decoder fine-tune steps"},
        "data": "synthetic", "codec": "bc7" if codec else "bc4", "border": border, "models": M,
        "train_params": int(tr.n_params),
        "train_ms_per_step": train_ms / n_steps, "train_samples_per_s": M * BATCH * n_steps / (train_ms * 1e-3),
        "loss_curve": losses, "decode": out,
        "bits_per_texel": bits_per_texel_hybrid(TILE, TILE, frames, s_uvt, 12, (64, 64, 24), hidden, _bits(codec)),
    }
