#!/usr/bin/env python3
"""Benchmark of the NDGI decode hot path on one MI355X.

One step = the 4096x4096 workload: decode every texel of the atlas at one time t through
the persistent page decoder (1024 pages of 128^2), then 16,000,000 uniformly random
(u, v, t) queries, both on the FP16 MFMA path.  Inputs are resident in device memory
before the timed region.  The same JSON line also reports the FP32 path on the same
step, a 32-map virtual-texturing frame (p50 / p99), the training step with BC simulation
(1024^2 x 24, 2^18 samples), the roofline of the dominant kernel and the CPU oracle
timed on a bounded sample, and the paper's own hybrid layout (a 1024^2 lightmap of 64
per-tile models, each profile of Table 3) beside the paper's Table 5 latencies.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload c2|c5|hfit|hmap] [--hybrid-only]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "decoded texels/s (BC fetch+interp+MLP), FP16 MFMA vs FP32; train texels/s"
HBM_PEAK_GBS = 8000.0
W = H = 4096
GW = GH = 1024
T = 24
N_RANDOM = 16_000_000
PAGE = 128
# algorithmic bytes per texel of the frame decode: 4 B of BC4 blocks (8 ch x 8 B per 16
# texels), 2 B of FP16 grid (the two keys' 1024^2 x 8 x 2 B spread over 4096^2 texels),
# 6 B of FP16 RGB out
FRAME_BYTES_PER_TEXEL = 4.0 + 2.0 + 6.0
# random queries: every BC4 block and every grid node of all 24 keys is read at least once
# (compulsory), plus 12 B of query in and 6 B of RGB out per query
RANDOM_COMPULSORY_BYTES = (W * H // 16 * 8 * 8) + (T * GH * GW * 8 * 2) + N_RANDOM * (12 + 6)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Sources of the kernels whose HBM byte counters profiles/traffic.json records (the frame
# and random-access decode of the step), with the ABI header and the build flags.
DIGEST_SOURCES = ("csrc/device.hpp", "csrc/internal.hpp", "csrc/decode.hip", "csrc/binned.hip", "build.py")


def source_digest() -> str:
    """sha256 over DIGEST_SOURCES and include/ndgi.h: the identity of the code whose HBM byte
    counters profiles/traffic.json records."""
    import hashlib
    h = hashlib.sha256()
    files = [os.path.join(ROOT, "paper_2604_12625_amd", f) for f in DIGEST_SOURCES]
    files += [os.path.join(ROOT, "include", "ndgi.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel_key: str):
    """HBM bytes per launch of `kernel_key` from the committed byte-counter summary, or None
    when there is none or the sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("sources_sha256") != source_digest():
        return None
    k = rec.get("per_launch", {}).get(kernel_key)
    return None if k is None else k["traffic_bytes"]


class Timer:
    """HIP events on torch's current stream (the stream every launch below uses)."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = []

    def start(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def stop(self, e0):
        e1 = self.torch.cuda.Event(enable_timing=True)
        e1.record()
        self.pairs.append((e0, e1))

    def ms(self):
        return [a.elapsed_time(b) for a, b in self.pairs]


def c2_inputs(torch, N, I):
    m = I.random_model_torch(W, H, GW, GH, T, seed=2, device="cuda")
    dm = N.DeviceModel(W, H, GW, GH, T, m["bc4"], m["grid"], m["mlp"])
    marr = N.models_array([dm])
    t = 0.3711
    py, px = torch.meshgrid(torch.arange(H // PAGE), torch.arange(W // PAGE), indexing="ij")
    px = px.reshape(-1).numpy()
    py = py.reshape(-1).numpy()
    n_pages = px.size
    rq = N.page_requests([0] * n_pages, px, py, [t] * n_pages, py * PAGE * W + px * PAGE)
    nreq = torch.tensor([n_pages], dtype=torch.int32, device="cuda")
    q = I.uniform_queries_torch(N_RANDOM, seed=3, device="cuda")
    return dm, marr, rq, nreq, n_pages, q


def run_c2(args, torch, N, I, ctx):
    from paper_2604_12625_amd.autotune import tune_pages
    dm, marr, rq, nreq, n_pages, q = c2_inputs(torch, N, I)
    plain = N.Context(0)   # no reserved workspace: ndgi_decode's query-order pass
    out = {}
    tune_dst = torch.empty((W * H, 3), dtype=torch.float16, device="cuda")
    shape, timings = tune_pages(ctx, lambda: ctx.decode_pages(marr, 1, rq, nreq, n_pages, PAGE, tune_dst, W,
                                                              N.PREC_F16), "frame4096", use_cache=False)
    del tune_dst
    log(f"autotuned page launch (tile_w, tile_h, waves/CU) = {shape}")
    out["launch_shape"] = list(shape)
    for prec, name in ((N.PREC_F16, "f16"), (N.PREC_F32, "f32")):
        dt = torch.float16 if prec == N.PREC_F16 else torch.float32
        frame = torch.empty((W * H, 3), dtype=dt, device="cuda")
        rnd = torch.empty((N_RANDOM, 3), dtype=dt, device="cuda")
        # workspaces are reserved once, outside the timed region: the context's for ndgi_decode
        # (which then takes the binned kernels), a caller buffer for ndgi_decode_binned
        ws = torch.empty(ctx.binned_workspace_bytes(dm, N_RANDOM), dtype=torch.uint8, device="cuda")
        ctx.reserve_decode(dm, N_RANDOM)

        def random_leg():
            if args.random_path == "decode":
                ctx.decode(dm, q, prec, out=rnd)
            elif args.random_path == "binned":
                ctx.decode_binned(dm, q, prec, out=rnd, workspace=ws)
            else:
                plain.decode(dm, q, prec, out=rnd)

        def step(tf=None, tr=None):
            e = tf.start() if tf else None
            ctx.decode_pages(marr, 1, rq, nreq, n_pages, PAGE, frame, W, prec)
            if tf:
                tf.stop(e)
                e = tr.start()
            random_leg()
            if tr:
                tr.stop(e)

        steps = args.steps if prec == N.PREC_F16 else max(3, args.steps // 4)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        tf, tr = Timer(torch), Timer(torch)
        t0 = time.perf_counter()
        for _ in range(steps):
            step(tf, tr)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        fm, rm = tf.ms(), tr.ms()
        out[name] = dict(steps=steps, wall_s=wall, frame_ms=sum(fm) / len(fm), random_ms=sum(rm) / len(rm))
        # the query-order pass on the same queries (a context with no reservation), for
        # comparison (not in the step)
        to = Timer(torch)
        for _ in range(3):
            e = to.start()
            plain.decode(dm, q, prec, out=rnd)
            to.stop(e)
        torch.cuda.synchronize()
        out[name]["random_direct_ms"] = sorted(to.ms())[1]
        log(f"C2 {name}: {1e3 * wall / steps:.3f} ms/step (frame {out[name]['frame_ms']:.3f} ms, "
            f"random {out[name]['random_ms']:.3f} ms)")
        del frame, rnd, ws
    ctx.reserve_decode(None, 0)
    plain.close()
    return out, (dm, q)


# Decoder work per texel (2 (16 x 32 + 32 x 32 + 32 x 3) flop) and the dense FP16 MFMA peak.
MLP_FLOP_PER_TEXEL = 3264
MFMA_F16_PEAK_TFLOPS = 2500.0


def vt_frame_bytes(sides, mi, px, py, t, page=PAGE):
    """Compulsory HBM bytes of one VT frame: the BC4 blocks of every distinct (map, page),
    the 8-channel FP16 grid nodes of every distinct (map, page, key) window the page's
    texel centres interpolate (keys k0 and k1 of each request's t, periodic over T), and the
    6-byte RGB of every requested texel."""
    import numpy as np
    mi, px, py = np.asarray(mi), np.asarray(px), np.asarray(py)
    pages = set(zip(mi.tolist(), px.tolist(), py.tolist()))
    tau = np.asarray(t, np.float64) * T
    k0 = np.floor(tau).astype(np.int64) % T
    k1 = (k0 + 1) % T
    windows = set(zip(mi.tolist(), px.tolist(), py.tolist(), k0.tolist())) | \
        set(zip(mi.tolist(), px.tolist(), py.tolist(), k1.tolist()))
    total = len(pages) * (page * page // 16) * 64
    gp = page // 4                       # grid nodes per page side (grid at a quarter of the texels)
    for m, x, y, _ in windows:
        G = int(sides[m]) // 4
        nx = min(G - 1, gp * x + gp) - max(0, gp * x - 1) + 1
        ny = min(G - 1, gp * y + gp) - max(0, gp * y - 1) + 1
        total += nx * ny * 16
    return total + len(mi) * page * page * 6


def run_c1(args, torch, N, I, ctx, reps=50):
    """The tiny parity configuration: 64 x 64 map, 16 x 16 x 8 grid, all 4096 texel centres at
    8 times (32,768 queries); decode latency of one call, FP32 and FP16."""
    import numpy as np
    m = I.random_model(64, 64, 16, 16, 8, np.float32, np.float32, config=1)
    dm = N.DeviceModel.from_numpy(m)
    ts = I.rng(1, I.P_QUERY).random(8, dtype=np.float32)
    q = torch.from_numpy(I.texel_centre_queries(64, 64, ts)).cuda()
    out = {"queries": int(q.shape[0])}
    for prec, name in ((N.PREC_F32, "f32"), (N.PREC_F16, "f16")):
        o = ctx.decode(dm, q, prec)
        tm = Timer(torch)
        for _ in range(reps):
            e = tm.start()
            ctx.decode(dm, q, prec, out=o)
            tm.stop(e)
        torch.cuda.synchronize()
        ms = sorted(tm.ms())
        out[f"{name}_latency_us_p50"] = 1e3 * ms[reps // 2]
        out[f"{name}_latency_us_p99"] = 1e3 * ms[min(reps - 1, int(round(0.99 * (reps - 1))))]
    log(f"C1: FP32 {out['f32_latency_us_p50']:.1f} us, FP16 {out['f16_latency_us_p50']:.1f} us per call")
    return out


def run_c3(args, torch, N, I, ctx, frames=110, warm=10):
    """32 maps, 2000 page requests per frame (Zipf 1.1), one graph replay per frame."""
    import numpy as np
    from paper_2604_12625_amd.autotune import tune_pages
    g = I.rng(3, I.P_MODEL)
    sides = I.vt_map_sides(32, g)
    models = []
    for i, s in enumerate(sides):
        m = I.random_model_torch(int(s), int(s), int(s) // 4, int(s) // 4, T, seed=1000 + i, device="cuda")
        models.append(N.DeviceModel(int(s), int(s), int(s) // 4, int(s) // 4, T, m["bc4"], m["grid"], m["mlp"]))
    marr = N.models_array(models)
    n_req, per_row = 2000, 50
    pitch = per_row * PAGE
    dst = torch.empty((((n_req + per_row - 1) // per_row) * PAGE * pitch, 3), dtype=torch.float16, device="cuda")
    offs = np.array([(i // per_row) * PAGE * pitch + (i % per_row) * PAGE for i in range(n_req)], dtype=np.int64)
    all_rq, frame_bytes = [], []
    for f in range(frames):
        mi, px, py, t = I.vt_requests(sides, n_req, I.rng(3, I.P_REQ, f))
        all_rq.append(N.page_requests(mi, px, py, t, offs))
        frame_bytes.append(vt_frame_bytes(sides, mi, px, py, t))
    rq = torch.empty_like(all_rq[0])
    nreq = torch.tensor([n_req], dtype=torch.int32, device="cuda")
    rq.copy_(all_rq[0])
    shape, _ = tune_pages(ctx, lambda: ctx.decode_pages(marr, len(models), rq, nreq, n_req, PAGE, dst, pitch,
                                                        N.PREC_F16), "vt32", use_cache=False)
    log(f"autotuned VT launch (tile_w, tile_h, waves/CU) = {shape}")
    tm = Timer(torch)
    texels = n_req * PAGE * PAGE
    for f in range(frames):
        rq.copy_(all_rq[f])
        e = tm.start()
        ctx.decode_pages(marr, len(models), rq, nreq, n_req, PAGE, dst, pitch, N.PREC_F16, graph=True)
        tm.stop(e)
    torch.cuda.synchronize()
    times = tm.ms()[warm:]
    ms = sorted(times)
    p50 = ms[len(ms) // 2]
    p99 = ms[min(len(ms) - 1, int(round(0.99 * (len(ms) - 1))))]
    log(f"C3 VT frame: p50 {p50:.3f} ms, p99 {p99:.3f} ms ({texels / p50 / 1e6:.1f} G texels/s at p50)")
    assert ctx.error_flags() == 0
    # roofline per frame: its compulsory bytes at the HBM peak against its decoder flops at
    # the FP16 MFMA peak; the median over the timed frames of (bound time / frame time)
    fb = frame_bytes[warm:]
    t_hbm = [b / (HBM_PEAK_GBS * 1e9) for b in fb]
    t_mfma = texels * MLP_FLOP_PER_TEXEL / (MFMA_F16_PEAK_TFLOPS * 1e12)
    fracs = sorted(max(th, t_mfma) / (tt * 1e-3) for th, tt in zip(t_hbm, times))
    mean_b = sum(fb) / len(fb)
    bound = "hbm" if sum(t_hbm) / len(t_hbm) >= t_mfma else "mfma"
    rl = dict(bound=bound, peak=HBM_PEAK_GBS if bound == "hbm" else MFMA_F16_PEAK_TFLOPS,
              unit="GB/s" if bound == "hbm" else "TFLOP/s", traffic=None, kernel="k_decode_tiles (graph replay)",
              bytes_per_launch=mean_b, flop_per_launch=texels * MLP_FLOP_PER_TEXEL)
    rl["achieved"] = (mean_b / (p50 * 1e-3) / 1e9 if bound == "hbm"
                      else texels * MLP_FLOP_PER_TEXEL / (p50 * 1e-3) / 1e12)
    rl["frac"] = fracs[len(fracs) // 2]
    return dict(p50_ms=p50, p99_ms=p99, texels_per_frame=texels, launch_shape=list(shape),
                maps=[int(s) for s in sides], roofline=rl,
                bound_us=dict(hbm=1e6 * sum(t_hbm) / len(t_hbm), mfma=1e6 * t_mfma))


# Decode latency of a 1024 x 1024 lightmap reported for the paper's profiles on an RTX 4060
# (Table 5), quoted beside the measurement as context (other hardware, not a target).
PAPER_TABLE5_MS = {"L": 0.201, "M": 0.203, "M.64": 0.314}


def run_hybrid(args, torch, N, I, ctx, reps=30, warm=5):
    """The paper's own layout and decoder: a 1024 x 1024 lightmap as 64 per-tile models of
    128 x 128 texels (F_uv 128^2 x 4 and F_uvt side^2 x 12 x 4 as BC7 blocks, the paper's
    format, or as four BC4 blocks per footprint; F_ut / F_vt 64 x 24 x 2 8-bit; 26 key
    times), all 64 pages decoded at one t in one persistent launch, for each profile of
    Table 3, both codecs and both precisions; and profile M with the 4-texel mirrored tile
    border of the paper's VT storage (64 regions of 136^2).  The BC7 blocks are mode 6, the
    mode the export of the paper's recipe writes for all but a few blocks in 10^4; one more
    row (M.bc7mix) draws modes 4, 5 and 6 per block, the decode's divergent worst case."""
    import numpy as np
    out = {}
    idx = np.arange(64)
    rows = (("L", 1, 0, (6,)), ("M", 1, 0, (6,)), ("H", 1, 0, (6,)), ("M.64", 1, 0, (6,)), ("L", 0, 0, ()),
            ("M", 0, 0, ()), ("H", 0, 0, ()), ("M.64", 0, 0, ()), ("M", 1, 4, (6,)), ("M", 1, 0, (4, 5, 6)))
    for prof, codec, border, modes in rows:
        R = 128 + 2 * border
        pitch = 8 * R
        offs = ((idx // 8) * R * pitch + (idx % 8) * R).astype(np.int64)
        models = [N.HybridModel.from_numpy(I.random_hybrid_model(profile=prof, config=6, index=i, codec=codec,
                                                                 bc7_modes=modes or (6,)))
                  for i in range(64)]
        marr = N.models_array(models)
        rq = N.page_requests(idx.astype(np.int32), np.zeros(64, np.int32), np.zeros(64, np.int32),
                             np.full(64, 0.4375, np.float32), offs)
        nreq = torch.tensor([64], dtype=torch.int32, device="cuda")
        row = {"codec": "bc7" if codec else "bc4", "border": border, "texels": 64 * R * R}
        for prec, name in ((N.PREC_F16, "f16"), (N.PREC_F32, "f32")):
            dst = torch.empty((pitch * pitch, 3), dtype=torch.float16 if prec == N.PREC_F16 else torch.float32,
                              device="cuda")
            widths = 2 if I.HYBRID_PROFILES[prof][1] == 64 else 1

            def call():
                ctx.hybrid_decode_pages(marr, 64, rq, nreq, 64, 128, dst, pitch, prec, widths=widths, border=border)
            for _ in range(warm):
                call()
            tm = Timer(torch)
            for _ in range(reps):
                e = tm.start()
                call()
                tm.stop(e)
            torch.cuda.synchronize()
            ms = sorted(tm.ms())[reps // 2]
            row[f"{name}_ms"] = ms
            row[f"{name}_texels_per_s"] = 64 * R * R / (ms * 1e-3)
        if prof in PAPER_TABLE5_MS and not border and len(modes) < 2:
            row["paper_rtx4060_ms"] = PAPER_TABLE5_MS[prof]
        # roofline of the FP16 launch: compulsory bytes of one decode at one t (every F_uv
        # block, the two F_uvt slices and the two F_ut / F_vt time columns around t, the
        # decoder) plus the FP16 RGB out, against the decoder's flops at the FP16 MFMA peak
        d = models[0].desc
        hid = d.hidden
        blk = 1 if codec else 2                                      # bytes per texel of a BC7 / 4 x BC4 map
        in_b = 64 * (d.W * d.H * blk + 2 * d.Gu * d.Gv * blk + 2 * 2 * (d.U + d.V) + 2 * I.hybrid_mlp_size(hid))
        flop = 64 * R * R * 2 * (16 * hid + hid * hid + 3 * hid)
        t_h, t_m = (in_b + 64 * R * R * 6) / (HBM_PEAK_GBS * 1e9), flop / (MFMA_F16_PEAK_TFLOPS * 1e12)
        row["roofline_f16"] = dict(bound="hbm" if t_h >= t_m else "mfma", bytes_per_launch=in_b + 64 * R * R * 6,
                                   flop_per_launch=flop, frac=max(t_h, t_m) / (row["f16_ms"] * 1e-3),
                                   achieved=(in_b + 64 * R * R * 6) / (row["f16_ms"] * 1e-3) / 1e9, unit="GB/s",
                                   peak=HBM_PEAK_GBS, traffic=None)
        key = prof + ("" if codec else ".bc4") + (f".border{border}" if border else "") + (".bc7mix" if len(modes) > 1 else "")
        log(f"hybrid 1024^2 {key}: FP16 {row['f16_ms'] * 1e3:.1f} us, FP32 {row['f32_ms'] * 1e3:.1f} us")
        out[key] = row
    assert ctx.error_flags() == 0
    return out


def run_hybrid_train(args, torch, N, I, ctx, steps=10, warm=3):
    """The paper's production training step: 64 tile models of 128^2 (profile M, BC7), 4096
    samples per model (the paper's batch), one fused phase-1 step (forward on the continuous
    endpoint / weight maps with noise, loss, backward, Adam) per launch pair; samples drawn
    before the timed region."""
    from paper_2604_12625_amd.train import HybridTrainer, hybrid_normalize_target
    keys = I.lightmap_key_times(I.rng(6, I.P_MODEL, 1))
    frames, M, Bm = len(keys), 64, 4096
    inits = [I.hybrid_train_init(128, 128, "M", frames, keys, I.rng(7, I.P_INIT, m), codec=1) for m in range(M)]
    tr = HybridTrainer(ctx, inits, lr_feat=1e-3, lr_mlp=1e-3, seed=1, per_model=Bm)
    scene = I.light_scene(1024, 1024, I.rng(7, I.P_TARGET))
    full = torch.stack([I.scene_frame_torch(scene, float(t), device="cuda").to(torch.float16) for t in keys])
    tiles = full.view(frames, 8, 128, 8, 128, 3).permute(1, 3, 0, 2, 4, 5).reshape(M * frames, 128, 128, 3)
    tgt, _ = hybrid_normalize_target(ctx, tiles.contiguous().view(torch.int16), 2.2)
    smp = [I.train_samples_torch(M * Bm, 128, 128, frames, seed=80_000 + i, border=4) for i in range(warm + steps)]
    flags = N.HTRAIN_NOISE
    for i in range(warm):
        tr.step(smp[i], tgt, flags)
    torch.cuda.synchronize()
    tm = Timer(torch)
    for i in range(steps):
        e = tm.start()
        tr.step(smp[warm + i], tgt, flags)
        tm.stop(e)
    torch.cuda.synchronize()
    ms = sorted(tm.ms())[steps // 2]
    log(f"hybrid train, 64 tile models x 4096 samples: {ms:.3f} ms/step ({M * Bm / ms / 1e3:.1f} M samples/s)")
    # algorithmic bytes of a step: per sample 4 B of index and 6 B of target, FP32 reads of the
    # parameters it touches (F_uv footprint: 8 endpoints + 1 weight; F_uvt: 4 taps x 2 slices x
    # (8 endpoints + 1 weight); F_ut / F_vt: 2 planes x 2 positions x 2 times x 2 channels) and
    # the read-modify-write of their gradients; dense Adam at 32 B per parameter
    touched = (8 + 1) + 4 * 2 * (8 + 1) + 2 * 2 * 2 * 2
    step_bytes = M * Bm * (10 + 3 * 4 * touched) + int(tr.n_params) * 32
    rl = dict(bound="hbm", achieved=step_bytes / (ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s", traffic=None,
              bytes_per_launch=step_bytes, kernel="ndgi_hybrid_train_step FUSED (k_hybrid_train, k_adam)")
    rl["frac"] = rl["achieved"] / HBM_PEAK_GBS
    return dict(ms_per_step=ms, samples_per_s=M * Bm / (ms * 1e-3), models=M, per_model=Bm, profile="M", codec="bc7",
                params=int(tr.n_params), loss=float(tr.loss.item()), roofline=rl)


def run_c4(args, torch, N, I, ctx, steps=None, warm=3):
    """Training step with BC simulation: 1024^2 x 24 target, 2^18 samples, Adam."""
    import numpy as np
    from paper_2604_12625_amd.train import Trainer
    Wt = Ht = 1024
    Gt = 256
    scene = I.light_scene(Wt, Ht, I.rng(4, I.P_TARGET))
    tgt = I.scene_target_torch(scene, T, device="cuda")
    mean = tgt.float().mean(dim=(0, 1, 2)).cpu().numpy()
    st = I.train_init(Wt, Ht, Gt, Gt, T, mean, I.rng(4, I.P_INIT))
    tr = Trainer(ctx, st, lr_feat=1e-2, lr_mlp=1e-3)
    tgt_bits = tgt.view(torch.int16)
    B = 1 << 18
    steps = steps or args.steps
    smp = [I.train_samples_torch(B, Wt, Ht, T, seed=4000 + i) for i in range(warm + steps)]
    for i in range(warm):
        tr.step(smp[i], tgt_bits)
    torch.cuda.synchronize()
    tm = Timer(torch)
    t0 = time.perf_counter()
    for i in range(steps):
        e = tm.start()
        tr.step(smp[warm + i], tgt_bits)
        tm.stop(e)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = sum(tm.ms()) / steps
    loss = float(tr.loss.item())
    log(f"C4 train: {ms:.3f} ms/step, {B / ms / 1e6:.3f} G samples/s, loss {loss:.4e}")
    # algorithmic bytes of a step: per sample 4 B of index, 6 B of target, 224 B of gathered
    # parameters (8 channels x (2 endpoints + 1 weight) + 4 grid nodes x 8 channels, FP32) and
    # 448 B of atomic read-modify-write on their gradients; dense Adam reads parameter,
    # gradient, m, v and writes all four (32 B per parameter)
    n_par = int(tr.n_params)
    step_bytes = B * (4 + 6 + 224 + 448) + n_par * 32
    rl = dict(bound="hbm", achieved=step_bytes / (ms * 1e-3) / 1e9, peak=HBM_PEAK_GBS, unit="GB/s", traffic=None,
              kernel="ndgi_train_step FUSED (k_train, partial-row reduction, k_adam)", bytes_per_launch=step_bytes)
    rl["frac"] = rl["achieved"] / HBM_PEAK_GBS
    tgt_np = tgt.cpu().numpy()
    oracle_state = ({kk: np.asarray(st[kk], np.float64) for kk in ("endpoints", "weights", "grid", "mlp")}
                    | {"dims": st["dims"]}, lambda x, y, k: tgt_np[k, y, x].astype(np.float64))
    return (dict(ms_per_step=ms, samples_per_s=B / (wall / steps), batch=B, params=n_par, loss=loss, roofline=rl),
            oracle_state)


def _host_cpu():
    """Cores this process may run on (capped at 16, the host share of one GPU here) and the CPU
    model."""
    cores = len(os.sched_getaffinity(0))
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return cores, min(cores, 16), model


_POOL_MODEL = None


def _pool_chunk(a):
    """Worker of the multi-process oracle: decode one chunk of the shared query array."""
    from threadpoolctl import threadpool_limits
    from oracle import ndgi_oracle as O
    model, qs, chunk = _POOL_MODEL
    with threadpool_limits(limits=1):
        O.decode(model, qs[a * chunk:(a + 1) * chunk])
    return chunk


def cpu_baseline(args, dm, q, seconds, c4_state=None):
    """The CPU oracle (FP64 numpy, as it stands) on bounded samples of the same workload on
    this host: (i) one process with BLAS pinned to 1 thread and (ii) worker processes over the
    host cores (forked from this process; they only run numpy), on the first 2^20 random
    queries; the frame subsample (2^20 texel centres at stride 16) and the C1 set in mode (i);
    and the training oracle's gradient on a 2^12-sample C4 batch."""
    import multiprocessing as mp
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import ndgi_oracle as O
    global _POOL_MODEL
    n_aff, n_use, cpu_model = _host_cpu()
    model = dict(W=W, H=H, Gw=GW, Gh=GH, T=T, bc4=dm.bc4.cpu().numpy(), grid=dm.grid.cpu().numpy(),
                 mlp=dm.mlp.cpu().numpy())
    qs = q[: 1 << 20].cpu().numpy()
    chunk = 1 << 15
    nchunks = (1 << 20) // chunk
    res = {}

    def timed(fn, budget):
        done, t0 = 0, time.perf_counter()
        while True:
            done += fn(done)
            if time.perf_counter() - t0 >= budget:
                return done, time.perf_counter() - t0

    with threadpool_limits(limits=1):
        # (i) random queries, one thread
        def rnd(done):
            a = (done // chunk) % nchunks
            O.decode(model, qs[a * chunk:(a + 1) * chunk])
            return chunk
        done, el = timed(rnd, 0.5 * seconds)
        res["random_1thread_queries_per_s"] = done / el
        # frame subsample: 2^20 texel centres at stride 16 (t of the frame), one thread
        sel = np.arange(0, W * H, 16)
        xs, ys = sel % W, sel // W
        tf = np.float64(np.float32(0.3711))

        def frame(done):
            a = (done // chunk) % nchunks
            xx, yy = xs[a * chunk:(a + 1) * chunk], ys[a * chunk:(a + 1) * chunk]
            O.decode_f64(model, (xx + 0.5) / W, (yy + 0.5) / H, np.full(xx.size, tf))
            return chunk
        done, el = timed(frame, 0.2 * seconds)
        res["frame_1thread_texels_per_s"] = done / el
        # C1 set (64^2 map, all texel centres at 8 times), one thread
        from paper_2604_12625_amd import inputs as I
        m1 = I.random_model(64, 64, 16, 16, 8, np.float32, np.float32, config=1)
        q1 = I.texel_centre_queries(64, 64, I.rng(1, I.P_QUERY).random(8, dtype=np.float32))
        t0 = time.perf_counter()
        O.decode(m1, q1)
        res["c1_1thread_s"] = time.perf_counter() - t0
        # training oracle: gradient of one 2^12-sample batch on the C4 state
        if c4_state is not None:
            st, tgt_fn = c4_state
            x, y, k = I.train_samples(1 << 12, 1024, 1024, T, I.rng(4, I.P_SAMPLES, 99))
            t0 = time.perf_counter()
            O.train_grads(st, x, y, k, tgt_fn(x, y, k))
            el = time.perf_counter() - t0
            res["train_1thread_us_per_sample"] = 1e6 * el / (1 << 12)
    # (ii) random queries over the host cores
    _POOL_MODEL = (model, qs, chunk)
    per = max(1, int(0.3 * seconds * res["random_1thread_queries_per_s"] / chunk))   # ~0.3 s-budget per worker
    jobs = [a % nchunks for a in range(per * n_use)]
    with mp.get_context("fork").Pool(n_use) as pool:
        t0 = time.perf_counter()
        done = sum(pool.map(_pool_chunk, jobs, chunksize=1))
        el = time.perf_counter() - t0
    _POOL_MODEL = None
    res["random_multiproc_queries_per_s"] = done / el
    return dict(value=res["random_multiproc_queries_per_s"], unit="texels/s", cores=n_use, kind="oracle",
                sample=f"{done} decodes cycling over the workload's first 2^20 uniform random queries (chunks of "
                       f"{chunk}) in {n_use} worker processes, FP64 numpy, BLAS 1 thread each, {el:.1f} s; host "
                       f"{cpu_model}, {n_aff} cores in this process's affinity",
                host_cpu=cpu_model, host_cores=n_aff, modes=res)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c2", choices=["c2", "c5", "hfit", "hmap"])
    ap.add_argument("--codec", default="both", choices=["both", "bc7", "bc4"],
                    help="block format of F_uv / F_uvt for the hfit and hmap workloads")
    ap.add_argument("--border", type=int, default=4, help="mirrored tile border (texels) of the hmap workload")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--random-path", default="decode", choices=["decode", "binned", "direct"],
                    help="decode of the random queries: ndgi_decode with a reserved context workspace (the "
                         "binned kernels; default), ndgi_decode_binned with a caller workspace, or ndgi_decode "
                         "without a reservation (one pass in query order)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true", help="skip the VT, hybrid and training legs")
    ap.add_argument("--hybrid-only", action="store_true", help="only the hybrid-layout decode leg")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus}); "
              "decode would shard by map ownership and per-tile training needs no communication, so each "
              "GPU would run this single-GPU path on its share", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2604_12625_amd import inputs as I
    from paper_2604_12625_amd import ndgi as N
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4, "launches": 5}))
        return
    ctx = N.Context(0)
    if args.hybrid_only:
        print(json.dumps({"hybrid_1024_tiles": run_hybrid(args, torch, N, I, ctx),
                          "hybrid_train_64_tiles": run_hybrid_train(args, torch, N, I, ctx)}), flush=True)
        return
    if args.workload == "hmap":
        from paper_2604_12625_amd.hybrid_fit import run_hfit_map
        print(json.dumps(run_hfit_map(args, torch, N, I, ctx)), flush=True)
        return
    if args.workload == "hfit":
        from paper_2604_12625_amd.hybrid_fit import run_hfit
        print(json.dumps(run_hfit(args, torch, N, I, ctx)), flush=True)
        return
    if args.workload == "c5":
        from paper_2604_12625_amd.large import run_c5
        print(json.dumps(run_c5(args, torch, N, I, ctx)), flush=True)
        return

    c2, (dm, q) = run_c2(args, torch, N, I, ctx)
    f16, f32 = c2["f16"], c2["f32"]
    texels_per_step = W * H + N_RANDOM
    ms_step = 1e3 * f16["wall_s"] / f16["steps"]
    value = texels_per_step / (f16["wall_s"] / f16["steps"])
    fp32_value = texels_per_step / (f32["wall_s"] / f32["steps"])

    frame_bytes = FRAME_BYTES_PER_TEXEL * W * H
    rl_frame = dict(bound="hbm", achieved=frame_bytes / (f16["frame_ms"] * 1e-3) / 1e9, peak=HBM_PEAK_GBS,
                    unit="GB/s", traffic=measured_traffic("frame_f16"),
                    kernel="k_decode_tiles (+ k_decode_pages<FP16> for items off the tile path)",
                    bytes_per_launch=frame_bytes)
    rl_frame["frac"] = rl_frame["achieved"] / HBM_PEAK_GBS
    rl_rand = dict(bound="hbm", achieved=RANDOM_COMPULSORY_BYTES / (f16["random_ms"] * 1e-3) / 1e9,
                   peak=HBM_PEAK_GBS, unit="GB/s",
                   traffic=measured_traffic("random_f16_" + ("direct" if args.random_path == "direct" else "binned")),
                   kernel=("k_decode_query<FP16>" if args.random_path == "direct" else
                           ("ndgi_decode with a reserved workspace -> " if args.random_path == "decode" else
                            "ndgi_decode_binned -> ") +
                           "k_bin_count, k_bin_colscan, k_bin_starts, k_bin_scatter, k_decode_binned_lds<FP16>"),
                   bytes_per_launch=RANDOM_COMPULSORY_BYTES)
    rl_rand["frac"] = rl_rand["achieved"] / HBM_PEAK_GBS
    # HBM rate the kernels actually drive: counter bytes per launch over the live launch time
    for rl, ms in ((rl_frame, f16["frame_ms"]), (rl_rand, f16["random_ms"])):
        rl["traffic_gbs"] = None if rl["traffic"] is None else rl["traffic"] / (ms * 1e-3) / 1e9
    dominant = rl_rand if f16["random_ms"] >= f16["frame_ms"] else rl_frame
    other = rl_frame if dominant is rl_rand else rl_rand

    res = {
        "metric": METRIC, "value": value, "unit": "texels/s", "n_gpus": 1, "steps": f16["steps"],
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f16", "data": "synthetic",
        "config": {"workload": "4096x4096 atlas, T=24 keys; 8-channel BC4 spatial map + 1024^2 x 24 x 8 FP16 grid; "
                               "16-32-32-3 FP16 decoder; step = full frame at one t (16,777,216 texels, 1024 "
                               "pages of 128^2) + 16,000,000 uniform random (u,v,t) queries",
                   "texels_per_step": texels_per_step, "precision": "FP16 MFMA, FP32 accumulate, FP16 out"},
        "roofline": dominant,
        "roofline_other": other,
        "fp16_frame_texels_per_s": W * H / (f16["frame_ms"] * 1e-3),
        "fp16_random_queries_per_s": N_RANDOM / (f16["random_ms"] * 1e-3),
        "fp32_texels_per_s": fp32_value,
        "fp32_frame_texels_per_s": W * H / (f32["frame_ms"] * 1e-3),
        "fp32_random_queries_per_s": N_RANDOM / (f32["random_ms"] * 1e-3),
        "fp16_over_fp32": value / fp32_value,
    }
    res["config"]["launch_shape"] = c2["launch_shape"]
    res["c1"] = run_c1(args, torch, N, I, ctx)
    c4_state = None
    if not args.headline_only:
        ctx3 = N.Context(0)
        res["vt_frame"] = run_c3(args, torch, N, I, ctx3)
        ctx3.close()
        res["hybrid_1024_tiles"] = run_hybrid(args, torch, N, I, ctx)
        res["hybrid_train_64_tiles"] = run_hybrid_train(args, torch, N, I, ctx)
        c4, c4_state = run_c4(args, torch, N, I, ctx)
        res["train_texels_per_s"] = c4["samples_per_s"]
        res["train"] = c4
    if not args.no_cpu_baseline:
        log("CPU oracle baseline ...")
        res["cpu_baseline"] = cpu_baseline(args, dm, q, args.cpu_seconds, c4_state)
    print(json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
