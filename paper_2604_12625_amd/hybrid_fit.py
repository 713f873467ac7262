"""Fit of the paper's hybrid layout to a temporal lightmap with its training recipe (Sec. 3.4,
Sec. 4), all on the GPU kernels, then export, decode and score.

Target: a 128 x 128 tile (the paper trains one model per VT tile) cut from the synthetic
1024^2 temporal lightmap, baked at 26 key times (24 hourly plus two around a light switch,
like the paper's sets), FP16.  Preprocessing: gamma 2.2 and per-frame, per-channel mean
normalisation.  Adam at the paper's learning rate 1e-3 and batch 2^12 texel samples.

Arms (the supplementary ablation compares the first two; both compress after training):
* with_bc_simulation (the paper's recipe): phase 1 trains F_uv / F_uvt as block endpoints
  and per-texel weights (Eq. 6-7, continuous) with U(-1/2, 1/2)/256 noise on the four sampled
  vectors; the export reconstructs the maps, quantises them to 8 bits and block-encodes them
  (ndgi_hybrid_encode); phase 2 fine-tunes the decoder on the frozen features of that
  compressed model (imported, DIRECT | QPLANES), i.e. under quantisation and BC compression.
* without_bc_simulation: phase 1 optimises the per-texel maps directly (DIRECT, noise as
  above), then the same export and phase 2.
* rounded_simulation (a variant the paper does not describe): phase 1 rounds endpoints and
  weights to the block grid with straight-through gradients (BCSIM | NOISE), the export is the
  exact encoding of the rounded parameters, phase 2 fine-tunes on BCSIM | QPLANES.
Each arm's model (BC7 blocks of modes 4-6 as in the paper, or BC4 blocks per channel; 8-bit planes,
FP16 decoder) is decoded for all 26 frames through the page decoder at their key times (FP16
and FP32 paths), restored, and scored by tiled PSNR (one 128^2 tile per frame).
"""
from __future__ import annotations

import sys
import time

import numpy as np

TILE = 128
GAMMA = 2.2
BATCH = 1 << 12
LR = 1e-3
ARMS = ("with_bc_simulation", "without_bc_simulation", "rounded_simulation")


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


def arm_flags(N, arm):
    """(phase-1 flags, export reconstruction flags, phase-2 flags) of an arm."""
    if arm == "with_bc_simulation":
        return N.HTRAIN_NOISE, 0, N.HTRAIN_DIRECT | N.HTRAIN_QPLANES
    if arm == "without_bc_simulation":
        return N.HTRAIN_DIRECT | N.HTRAIN_NOISE, N.HTRAIN_DIRECT, N.HTRAIN_DIRECT | N.HTRAIN_QPLANES
    return N.HTRAIN_BCSIM | N.HTRAIN_NOISE, N.HTRAIN_BCSIM, N.HTRAIN_BCSIM | N.HTRAIN_QPLANES


def arm_init(I, arm, codec, make):
    """Initial state(s) of an arm: make(codec) draws one; the direct arm keeps one value per
    texel and channel (the BC4 layout)."""
    return make(0 if arm == "without_bc_simulation" else codec)


def assemble(N, maps, rest):
    """A model with the blocks of `maps` and the planes and decoder of `rest`."""
    d = maps.desc
    a, b = maps.arrays, rest.arrays
    return N.HybridModel(d.W, d.H, d.Gu, d.Gv, d.S, d.U, d.V, d.Tt, d.hidden, a[0], a[1], b[2], b[3], a[4], b[5],
                         d.codec)


def train_arm(torch, N, ctx, arm, codec, inits, tgt, keys, frames, steps1, steps2, samples, per_model=0,
              lr=LR, seed=0):
    """Phase 1, export, phase 2 of one arm; returns (final models, info).  samples(i) gives
    step i's packed samples."""
    from .train import HybridTrainer, hybrid_import_models
    f1, fx, f2 = arm_flags(N, arm)
    M = len(inits)
    tr = HybridTrainer(ctx, inits, lr_feat=lr, lr_mlp=lr, seed=seed, per_model=per_model)
    losses = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record()
    for i in range(steps1):
        tr.step(samples(i), tgt, f1)
        if (i + 1) % 1000 == 0:
            losses.append((i + 1, float(tr.loss.item())))
    e1.record()
    e1.synchronize()
    ms1 = e0.elapsed_time(e1)
    if arm == "rounded_simulation":
        tr.set_lr(lr_feat=0.0)
        for i in range(steps1, steps1 + steps2):
            tr.step(samples(i), tgt, f2)
        final = [tr.export(N.DTYPE_F16, model=m) for m in range(M)]
        n_params = int(tr.n_params)
        enc_ms = 0.0
    else:
        torch.cuda.synchronize()
        te = time.perf_counter()
        enc = [tr.encode(fx, codec, N.DTYPE_F32, model=m) for m in range(M)]
        torch.cuda.synchronize()
        enc_ms = (time.perf_counter() - te) * 1e3
        n_params = int(tr.n_params)
        del tr
        tr2 = hybrid_import_models(ctx, enc, frames, lr_mlp=lr, seed=seed, per_model=per_model, keys=keys)
        for i in range(steps1, steps1 + steps2):
            tr2.step(samples(i), tgt, f2)
        final = [assemble(N, enc[m], tr2.encode(N.HTRAIN_DIRECT, codec, N.DTYPE_F16, model=m, maps=False))
                 for m in range(M)]
        tr = tr2
    torch.cuda.synchronize()
    losses.append((steps1 + steps2, float(tr.loss.item())))
    wall = time.perf_counter() - t0
    info = dict(train_ms_per_step=ms1 / steps1, wall_s=wall, encode_ms=enc_ms, loss_curve=losses,
                flags_phase1=int(f1), flags_export=int(fx), flags_phase2=int(f2), n_params=n_params)
    if codec == 1:
        info["bc7_mode_share"] = bc7_mode_share(torch, [a for m in final for a in m.arrays[:2]])
    return final, info


def bc7_mode_share(torch, block_arrays):
    """Share of BC7 blocks per mode (4, 5, 6) over device arrays of 16-byte blocks."""
    b0 = torch.cat([a.reshape(-1, 16)[:, 0] for a in block_arrays]).to(torch.int32)
    n = max(int(b0.numel()), 1)
    return {str(m): int(((b0 & ((2 << m) - 1)) == (1 << m)).sum().item()) / n for m in (4, 5, 6)}


def score(torch, N, ctx, models, means, target_tiles, keys, border=0):
    """Tiled PSNR of the decode (FP16 and FP32 paths) of every model at every key time against
    its target tile [M][frames][TILE][TILE][3]; with a border the decoded regions are
    (TILE + 2 border)^2 and the interiors are scored."""
    from .train import hybrid_restore
    M, frames = len(models), len(keys)
    R = TILE + 2 * border
    marr = N.models_array(models)
    mi = np.repeat(np.arange(M), frames).astype(np.int32)
    fi = np.tile(np.arange(frames), M)
    rq = N.page_requests(mi, np.zeros(M * frames, np.int32), np.zeros(M * frames, np.int32),
                         np.asarray(keys, np.float32)[fi], (np.arange(M * frames) * R * R).astype(np.int64))
    nreq = torch.tensor([M * frames], dtype=torch.int32, device="cuda")
    width = 2 if models[0].desc.hidden == 64 else 1
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
        tt = target_tiles.view(M * frames, TILE, TILE, 3)
        stats = []
        for k in range(M * frames):
            rec = hybrid_restore(ctx, inner[k * TILE * TILE:(k + 1) * TILE * TILE], means[k], GAMMA)
            stats.append(ctx.tile_stats(rec, tt[k].view(torch.int16), TILE, TILE, TILE))
        ps = ctx.psnr(torch.stack(stats), TILE, TILE, TILE)
        out[name] = dict(psnr_tiled_db=ps["tiled"], psnr_global_db=ps["global"],
                         psnr_tile_p10_db=ps["p10"], psnr_tile_min_db=ps["min"],
                         decode_all_frames_ms=ev0.elapsed_time(ev1))
    assert ctx.error_flags() == 0
    return out


def _codecs(args):
    c = getattr(args, "codec", "both")
    return {"bc4": (0,), "bc7": (1,), "both": (1, 0)}[c]


def _bits(codec):
    return 8 if codec == 1 else 16     # F_uv / F_uvt bits per texel: one BC7 block or four BC4 blocks


def bits_per_texel_hybrid(W, H, frames, side, slices, plane, hidden, uv_bits_per_texel):
    """Stored bits per texel per frame of a hybrid model: F_uv and the F_uvt slices at
    `uv_bits_per_texel` (16 for four BC4 channels, 8 for the paper's BC7), 8-bit planes,
    FP16 decoder."""
    U, V, Tt = plane
    mlp = hidden * 16 + hidden + hidden * hidden + hidden + 3 * hidden + 3
    bits = W * H * uv_bits_per_texel + side * side * slices * uv_bits_per_texel + (U + V) * Tt * 2 * 8 + mlp * 16
    return bits / (W * H * frames)


def run_hfit(args, torch, N, I, ctx, profile="M", steps1=4000, steps2=1000):
    """One tile, every arm, BC7 and BC4 (or the codec named)."""
    from .train import hybrid_normalize_target
    keys = I.lightmap_key_times(I.rng(6, I.P_MODEL, 1))
    frames = len(keys)
    target = tile_target(torch, I, keys)
    tgt, means = hybrid_normalize_target(ctx, target.view(torch.int16), GAMMA)
    side, hidden = I.HYBRID_PROFILES[profile]
    smp = torch.stack([I.train_samples_torch(BATCH, TILE, TILE, frames, seed=70_000 + i)
                       for i in range(steps1 + steps2)])
    results = {}
    for codec in _codecs(args):
        cname = "bc7" if codec else "bc4"
        runs = {}
        for arm in ARMS:
            init = arm_init(I, arm, codec, lambda c: I.hybrid_train_init(TILE, TILE, profile, frames, keys,
                                                                         I.rng(6, I.P_INIT), codec=c))
            models, info = train_arm(torch, N, ctx, arm, codec, [init], tgt, keys, frames, steps1, steps2,
                                     lambda i: smp[i])
            info["decode"] = score(torch, N, ctx, models, means, target[None], keys)
            runs[arm] = info
            _log(f"hybrid fit {profile} {cname} {arm}: {info['train_ms_per_step']:.3f} ms/step, "
                 f"PSNR FP16 {info['decode']['f16']['psnr_tiled_db']:.2f} dB, "
                 f"FP32 {info['decode']['f32']['psnr_tiled_db']:.2f} dB")
        results[cname] = dict(runs=runs, bits_per_texel=bits_per_texel_hybrid(TILE, TILE, frames, side, 12,
                                                                               (64, 64, 24), hidden, _bits(codec)))
    return {
        "metric": "hybrid-layout fit: tiled PSNR after export, train ms/step",
        "config": {"workload": f"one {TILE}x{TILE} tile of the synthetic 1024^2 temporal lightmap at 26 key times; "
                               f"profile {profile} (F_uvt {side}^2 x 12 x 4, hidden {hidden}); batch {BATCH}, Adam "
                               f"lr {LR}; {steps1} phase-1 steps, export (reconstruct, 8-bit, block-encode), "
                               f"{steps2} decoder fine-tune steps on the frozen compressed features; gamma 2.2 + "
                               "per-frame mean normalisation; arms: with / without BC simulation (supplementary "
                               "ablation), rounded simulation (variant)"},
        "data": "synthetic", "codecs": results,
    }


def run_hfit_map(args, torch, N, I, ctx, profile="M", side=1024, steps1=6000, steps2=2000):
    """The paper's production setting: a side x side lightmap as (side/128)^2 per-tile models,
    trained together in one launch per step (4096 samples per model), exported, and decoded
    for all 26 frames through the page decoder (one request per tile and frame, one launch).
    Tiles carry a mirrored border of `--border` texels (supplementary Virtual Texturing
    section; 4 by default): training samples are drawn over the mirror-padded tile and each
    decoded page is a (128 + 2 border)^2 region; PSNR is scored on the 128^2 interiors.  The
    paper's recipe and the ablation's direct arm, for BC7 and BC4 (or the codec named)."""
    from .train import hybrid_normalize_target
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
    border = int(getattr(args, "border", 4))
    s_uvt, hidden = I.HYBRID_PROFILES[profile]
    samples = lambda i: I.train_samples_torch(M * BATCH, TILE, TILE, frames, seed=90_000 + i, border=border)
    results = {}
    for codec in _codecs(args):
        cname = "bc7" if codec else "bc4"
        runs = {}
        for arm in ARMS[:2]:
            inits = [arm_init(I, arm, codec, lambda c: I.hybrid_train_init(TILE, TILE, profile, frames, keys,
                                                                           I.rng(7, I.P_INIT, m), codec=c))
                     for m in range(M)]
            models, info = train_arm(torch, N, ctx, arm, codec, inits, tgt, keys, frames, steps1, steps2, samples,
                                     per_model=BATCH, seed=1)
            info["train_samples_per_s"] = M * BATCH / (info["train_ms_per_step"] * 1e-3)
            info["decode"] = score(torch, N, ctx, models, means, tiles, keys, border=border)
            runs[arm] = info
            _log(f"hybrid map {cname} {arm}: {M} models, {info['n_params'] / 1e6:.2f} M parameters, "
                 f"{info['train_ms_per_step']:.3f} ms/step, encode {info['encode_ms']:.1f} ms, PSNR tiled FP16 "
                 f"{info['decode']['f16']['psnr_tiled_db']:.2f} dB (p10 {info['decode']['f16']['psnr_tile_p10_db']:.2f}),"
                 f" decode of {frames} frames {info['decode']['f16']['decode_all_frames_ms']:.3f} ms")
        results[cname] = dict(runs=runs, bits_per_texel=bits_per_texel_hybrid(TILE, TILE, frames, s_uvt, 12,
                                                                               (64, 64, 24), hidden, _bits(codec)))
    return {
        "metric": "hybrid-layout map fit: per-tile models trained together, tiled PSNR after export",
        "config": {"workload": f"{side}x{side} synthetic temporal lightmap at 26 key times as {M} tile models of "
                               f"{TILE}^2 with {border}-texel mirrored borders, profile {profile}; batch {BATCH} per "
                               f"model, Adam lr {LR}; {steps1} phase-1 steps, export, {steps2} decoder fine-tune "
                               "steps; arms with / without BC simulation"},
        "data": "synthetic", "border": border, "models": M, "codecs": results,
    }
