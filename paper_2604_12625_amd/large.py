"""Large training + decode run: fit a 4096 x 4096 atlas with 48 time keys under BC
simulation, export it, decode every texel of every key and score it.

Model: 8-channel BC4 spatial map (4096^2) + 1024^2 x 48 x 8 grid + 16-32-32-3 decoder;
target: the synthetic temporal lightmap (64 Gaussian lights with day cycles, 200 moving
occluders) at the 48 keys, FP16.  Training: batches of 2^20 random texel samples, L2
loss, Adam (1e-2 features, 1e-3 decoder), the decoded features recomputed in the
backward.  Afterwards the trained state is exported (BC4 blocks, FP16 grid and decoder)
and all 48 keys are decoded through the page decoder on the FP16 and the FP32 path;
tiled PSNR (128^2 tiles) against the target, bits per texel and throughputs are reported.
"""
from __future__ import annotations

import sys
import time

import numpy as np

W = H = 4096
GW = GH = 1024
T = 48
BATCH = 1 << 20
STEPS = 2000
PAGE = 128
TILE = 128


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def bits_per_texel(W, H, Gw, Gh, T, grid_bits=16, mlp_bits=16, mlp_size=1699):
    """Storage of the exported model per texel per key: BC4 at 4 bits per texel per
    channel (8 channels), the grid at grid_bits per value, the decoder at mlp_bits."""
    bits = W * H * 8 * 4 + Gw * Gh * T * 8 * grid_bits + mlp_size * mlp_bits
    return bits / (W * H * T)


def run_c5(args, torch, N, I, ctx, steps: int | None = None, batch: int = BATCH):
    from .train import Trainer
    steps = steps or STEPS
    t_setup = time.perf_counter()
    scene = I.light_scene(W, H, I.rng(5, I.P_TARGET))
    target = I.scene_target_torch(scene, T, device="cuda")            # [T][H][W][3] fp16
    mean = torch.zeros(3, dtype=torch.float64, device="cuda")
    for k in range(T):
        mean += target[k].double().sum(dim=(0, 1))
    mean = (mean / (T * H * W)).cpu().numpy()
    _log(f"C5 target ready ({time.perf_counter() - t_setup:.1f} s), mean RGB {mean}")
    tr = Trainer(ctx, I.train_init_torch(W, H, GW, GH, T, mean, seed=5), lr_feat=1e-2, lr_mlp=1e-3)
    tgt_bits = target.view(torch.int16)
    samples = torch.empty((steps, batch), dtype=torch.int32, device="cuda")
    for i in range(steps):
        samples[i] = I.train_samples_torch(batch, W, H, T, seed=5000 + i)
    torch.cuda.synchronize()
    _log(f"C5 setup {time.perf_counter() - t_setup:.1f} s; {tr.n_params / 1e6:.1f} M parameters")

    # training: every step is timed on the stream that runs it
    block = 250
    losses = []
    train_ms = 0.0
    for b0 in range(0, steps, block):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for i in range(b0, min(steps, b0 + block)):
            tr.step(samples[i], tgt_bits)
        e1.record()
        e1.synchronize()
        train_ms += e0.elapsed_time(e1)
        losses.append((min(steps, b0 + block), float(tr.loss.item())))
        _log(f"C5 step {losses[-1][0]}: loss {losses[-1][1]:.4e} ({train_ms / losses[-1][0]:.3f} ms/step)")
    del samples

    # export and decode all keys, FP16 and FP32 paths
    dm = tr.export(N.DTYPE_F16, N.DTYPE_F16)
    marr = N.models_array([dm])
    npx, npy = W // PAGE, H // PAGE
    py, px = np.meshgrid(np.arange(npy), np.arange(npx), indexing="ij")
    px, py = px.ravel(), py.ravel()
    n_req = T * px.size
    kk = np.repeat(np.arange(T), px.size)
    rq = N.page_requests(np.zeros(n_req, np.int32), np.tile(px, T).astype(np.int32),
                         np.tile(py, T).astype(np.int32), (kk / T).astype(np.float32),
                         (kk * W * H + np.tile(py * PAGE * W + px * PAGE, T)).astype(np.int64))
    nreq = torch.tensor([n_req], dtype=torch.int32, device="cuda")
    res = {}
    for prec, name in ((N.PREC_F16, "f16"), (N.PREC_F32, "f32")):
        dst = torch.empty((T * W * H, 3), dtype=torch.float16 if prec == N.PREC_F16 else torch.float32,
                          device="cuda")
        ctx.decode_pages(marr, 1, rq, nreq, n_req, PAGE, dst, W, prec)      # warm-up
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.decode_pages(marr, 1, rq, nreq, n_req, PAGE, dst, W, prec)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        assert ctx.error_flags() == 0
        stats = torch.stack([ctx.tile_stats(dst[k * W * H:(k + 1) * W * H], tgt_bits[k], W, H, TILE)
                             for k in range(T)])
        ps = ctx.psnr(stats, W, H, TILE)
        tiled, glob = ps["tiled"], ps["global"]
        db_all = ps["tile_db"].cpu().numpy().ravel()
        st = stats.cpu().numpy().reshape(-1, 3)
        rng_all = st[:, 0] - st[:, 1]                     # per tile: max - min of the target
        ok = ~np.isnan(db_all)
        db, rng = db_all[ok], rng_all[ok]
        # tile PSNR by the tile's dynamic range (the tiled mean weighs every tile equally, so
        # near-constant dark tiles with a tiny range dominate it)
        edges = [0.0, 0.01, 0.1, 1.0, 10.0, np.inf]
        by_range = []
        for lo, hi in zip(edges[:-1], edges[1:]):
            sel = (rng >= lo) & (rng < hi)
            if sel.any():
                by_range.append(dict(range_lo=lo, range_hi=None if np.isinf(hi) else hi, tiles=int(sel.sum()),
                                     mean_db=float(db[sel].mean()), p10_db=float(np.quantile(db[sel], 0.1))))
        res[name] = dict(decode_ms_all_keys=ms, decode_texels_per_s=T * W * H / (ms * 1e-3),
                         psnr_tiled_db=tiled, psnr_global_db=glob, psnr_tile_min_db=ps["min"],
                         psnr_tile_quantiles_db={q: float(np.quantile(db, q)) for q in (0.01, 0.1, 0.5, 0.9)},
                         psnr_by_tile_range=by_range, tiles_scored=ps["scored"], tiles=ps["tiles"])
        _log(f"C5 decode {name}: {ms:.2f} ms for {T} keys ({T * W * H / ms / 1e6:.1f} G texels/s), "
             f"PSNR tiled {tiled:.2f} dB, global {glob:.2f} dB")
        del dst
    train_s = train_ms * 1e-3
    return {
        "metric": "C5 large training + decode",
        "config": {"workload": "4096x4096 atlas, T=48; BC4 4096^2 x 8 + grid 1024^2 x 48 x 8; batch 2^20; "
                               f"{steps} Adam steps; decode of all 48 keys"},
        "data": "synthetic",
        "train_steps": steps, "batch": batch, "train_s": train_s,
        "train_ms_per_step": train_ms / steps,
        "train_texels_per_s": steps * batch / train_s,
        "loss_curve": losses,
        "bits_per_texel": bits_per_texel(W, H, GW, GH, T),
        "decode": res,
        "fp16_psnr_not_worse": res["f16"]["psnr_tiled_db"] >= res["f32"]["psnr_tiled_db"] - 0.01,
    }
