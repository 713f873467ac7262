"""Seeded synthetic inputs for the NDGI decode and training path.

This module only draws numbers and lays them out in the library's storage formats; it
contains none of the method's arithmetic (no block decoding, interpolation or MLP).
Both the HIP path (through tests and the benchmark) and the CPU reference use it.

Every generator takes a ``numpy.random.Generator`` made by :func:`rng`, whose stream is
``SeedSequence([seed, config, purpose, index])`` so that each workload, purpose (model,
queries, requests, target, samples) and step has its own independent stream.

The paper's lightmap dataset is not available; the synthetic workloads stand in for it:

* random models: BC4 blocks with uniformly random bytes (so both BC4 modes and every
  selector occur), a grid with values uniform in [-1, 1], He-normal decoder weights
  with zero biases;
* random hybrid models (the paper's four feature maps): random block bytes and 8-bit
  planes, He-normal weights with small uniform biases, key times of hourly bakes plus
  two around a light switch;
* queries: texel centres of a map at given times, or (u, v, t) uniform in [0, 1);
* virtual-texturing frames: maps with side 128 * round(2^U[1,5]) and page requests
  drawn Zipf(1.1) over a seeded ranking of the maps;
* a temporal lightmap target built from Gaussian lights with day-cycle intensity
  curves, shadowed by rectangles that move with time.
"""
from __future__ import annotations

import math

import numpy as np

N_CH = 8
HIDDEN = 32
N_IN = 16
N_OUT = 3
MLP_SIZE = HIDDEN * N_IN + HIDDEN + HIDDEN * HIDDEN + HIDDEN + N_OUT * HIDDEN + N_OUT

# purposes of the random streams
P_MODEL, P_QUERY, P_REQ, P_TARGET, P_SAMPLES, P_INIT = range(6)


def rng(config: int, purpose: int, index: int = 0, seed: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, config, purpose, index])))


# ------------------------------------------------------------------------------ models

def random_bc4(W: int, H: int, g: np.random.Generator) -> np.ndarray:
    """[H/4][W/4][8 channels][8 bytes] of uniformly random bytes."""
    assert W % 4 == 0 and H % 4 == 0
    return g.integers(0, 256, size=(H // 4, W // 4, N_CH, 8), dtype=np.uint8)


def random_grid(Gw: int, Gh: int, T: int, dtype, g: np.random.Generator) -> np.ndarray:
    """[T][Gh][Gw][8], values uniform in [-1, 1], stored in ``dtype`` (round to nearest)."""
    return g.uniform(-1.0, 1.0, size=(T, Gh, Gw, N_CH)).astype(np.float32).astype(dtype)


def he_normal_mlp(dtype, g: np.random.Generator) -> np.ndarray:
    """Packed [W1 32x16 | b1 | W2 32x32 | b2 | W3 3x32 | b3]; W ~ N(0, 2/fan_in), b = 0."""
    parts = []
    for (fo, fi) in ((HIDDEN, N_IN), (HIDDEN, HIDDEN), (N_OUT, HIDDEN)):
        parts.append(g.normal(0.0, math.sqrt(2.0 / fi), size=fo * fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32).astype(dtype)


def random_model(W: int, H: int, Gw: int, Gh: int, T: int, grid_dtype=np.float32,
                 mlp_dtype=np.float32, config: int = 0, index: int = 0) -> dict:
    g = rng(config, P_MODEL, index)
    return dict(W=W, H=H, Gw=Gw, Gh=Gh, T=T,
                bc4=random_bc4(W, H, g),
                grid=random_grid(Gw, Gh, T, grid_dtype, g),
                mlp=he_normal_mlp(mlp_dtype, g))


# ------------------------------------------------------------ hybrid feature maps
# The paper's own layout: F_uv (W x H x 4, block-compressed), F_ut (U x Tt x 2) and
# F_vt (V x Tt x 2) at 8 bits, F_uvt (Gu x Gv x S slices x 4, each slice
# block-compressed), a 16-h-h-3 decoder.  Profiles of a 128 x 128 tile model: F_uvt side
# 16 (L), 32 (M), 64 (H) with hidden width 16, and side 32 with width 64 (M.64); 12 slices;
# F_ut and F_vt 64 x 24.
HYBRID_IN = 16
HYBRID_PROFILES = {"L": (16, 16), "M": (32, 16), "H": (64, 16), "M.64": (32, 64)}


def hybrid_mlp_size(hidden: int) -> int:
    return hidden * HYBRID_IN + hidden + hidden * hidden + hidden + N_OUT * hidden + N_OUT


def hybrid_mlp(hidden: int, dtype, g: np.random.Generator) -> np.ndarray:
    """Packed [W1 h x 16 | b1 | W2 h x h | b2 | W3 3 x h | b3]; W ~ N(0, 2/fan_in),
    b ~ U[-0.1, 0.1]."""
    parts = []
    for (fo, fi) in ((hidden, HYBRID_IN), (hidden, hidden), (N_OUT, hidden)):
        parts.append(g.normal(0.0, math.sqrt(2.0 / fi), size=fo * fi))
        parts.append(g.uniform(-0.1, 0.1, size=fo))
    return np.concatenate(parts).astype(np.float32).astype(dtype)


def lightmap_key_times(g: np.random.Generator, hourly: int = 24, extra: int = 2) -> np.ndarray:
    """Key times of a day of baked lightmaps in [0, 1]: one per hour (h / hourly) plus
    ``extra`` keys around a light-switch time drawn inside an hour, 0.004 apart
    (strictly increasing, float32)."""
    s = (g.integers(2, hourly - 2) + g.uniform(0.3, 0.7)) / hourly
    extras = s + 0.004 * (np.arange(extra) - (extra - 1) / 2.0)
    return np.sort(np.concatenate([np.arange(hourly) / hourly, extras])).astype(np.float32)


def random_bc7m6(shape, g: np.random.Generator) -> np.ndarray:
    """Random BC7 mode-6 blocks [*shape][16]: uniform bytes with the mode bits set (bits 0..6
    of byte 0 = 1000000b; bit 7 belongs to the first endpoint value)."""
    b = g.integers(0, 256, size=tuple(shape) + (16,), dtype=np.uint8)
    b[..., 0] = (b[..., 0] & 0x80) | 0x40
    return b


def random_bc7(shape, g: np.random.Generator, modes=(4, 5, 6)) -> np.ndarray:
    """Random BC7 blocks [*shape][16] of the given modes (drawn uniformly per block): uniform
    bytes with the mode bits of byte 0 set (mode m: bits 0..m-1 clear, bit m set)."""
    b = g.integers(0, 256, size=tuple(shape) + (16,), dtype=np.uint8)
    m = np.asarray(modes)[g.integers(0, len(modes), size=tuple(shape))]
    keep = (0xFF << (m + 1)) & 0xFF
    b[..., 0] = ((b[..., 0] & keep) | (1 << m)).astype(np.uint8)
    return b


def random_hybrid_model(W: int = 128, H: int = 128, profile: str = "M", slices: int = 12,
                        plane=(64, 64, 24), mlp_dtype=np.float16, keys: bool = True,
                        config: int = 0, index: int = 0, uvt_side=None, codec: int = 0,
                        bc7_modes=(4, 5, 6)) -> dict:
    """A hybrid model with uniformly random block bytes and 8-bit planes.

    ``plane`` = (U, V, Tt): F_ut is [Tt][U][2] and F_vt is [Tt][V][2] (uint8);
    F_uv is [H/4][W/4][4][8] and F_uvt is [S][Gv/4][Gu/4][4][8] BC4 bytes (codec 0), or
    one 16-byte BC7 block per footprint (codec 1) of a mode drawn uniformly from
    ``bc7_modes``.  ``keys`` attaches a non-uniform key-time table (:func:`lightmap_key_times`)."""
    side, hidden = HYBRID_PROFILES[profile]
    Gu, Gv = (side, side) if uvt_side is None else uvt_side
    U, V, Tt = plane
    g = rng(config, P_MODEL, index)
    assert W % 4 == 0 and H % 4 == 0 and Gu % 4 == 0 and Gv % 4 == 0

    def blocks(shape):
        return random_bc7(shape, g, bc7_modes) if codec == 1 else g.integers(0, 256, size=tuple(shape) + (4, 8),
                                                                       dtype=np.uint8)

    return dict(
        W=W, H=H, Gu=Gu, Gv=Gv, S=slices, U=U, V=V, Tt=Tt, hidden=hidden, codec=codec,
        fuv=blocks((H // 4, W // 4)),
        fuvt=blocks((slices, Gv // 4, Gu // 4)),
        fut=g.integers(0, 256, size=(Tt, U, 2), dtype=np.uint8),
        fvt=g.integers(0, 256, size=(Tt, V, 2), dtype=np.uint8),
        keys=lightmap_key_times(g) if keys else np.zeros(0, np.float32),
        mlp=hybrid_mlp(hidden, mlp_dtype, g),
    )


def hybrid_train_init(W: int, H: int, profile: str, frames: int, keys, g: np.random.Generator,
                      slices: int = 12, plane=(64, 64, 24), codec: int = 0) -> dict:
    """Initial trainable hybrid state (float32): endpoints e1 ~ U[0, 0.5), e2 ~ U[0.5, 1],
    weights and planes ~ U[0, 1], He-normal decoder with zero biases except b3 = 1 (the
    normalised target has mean 1 in every channel)."""
    side, hidden = HYBRID_PROFILES[profile]
    U, V, Tt = plane

    def ep(shape):
        return np.stack([g.uniform(0.0, 0.5, shape), g.uniform(0.5, 1.0, shape)], axis=-1).astype(np.float32)

    mlp = hybrid_mlp(hidden, np.float32, g)
    o1 = hidden * HYBRID_IN                     # b1
    o2 = o1 + hidden + hidden * hidden          # b2
    mlp[o1:o1 + hidden] = 0.0
    mlp[o2:o2 + hidden] = 0.0
    mlp[-3:] = 1.0                              # b3
    cw = () if codec == 1 else (4,)     # one weight per texel (BC7) or per texel and channel (BC4)
    return dict(dims=dict(W=W, H=H, Gu=side, Gv=side, S=slices, U=U, V=V, Tt=Tt, hidden=hidden, frames=frames,
                          keys=np.asarray(keys, dtype=np.float32), codec=codec),
                fuv_ep=ep((H // 4, W // 4, 4)), fuv_w=g.uniform(0, 1, (H, W) + cw).astype(np.float32),
                fuvt_ep=ep((slices, side // 4, side // 4, 4)),
                fuvt_w=g.uniform(0, 1, (slices, side, side) + cw).astype(np.float32),
                fut=g.uniform(0, 1, (Tt, U, 2)).astype(np.float32), fvt=g.uniform(0, 1, (Tt, V, 2)).astype(np.float32),
                mlp=mlp)


# ----------------------------------------------------------------------------- queries

def texel_centre_queries(W: int, H: int, ts) -> np.ndarray:
    """All texel centres ((x+0.5)/W, (y+0.5)/H) of a W x H map at each t: [len(ts)*H*W][3] f32."""
    y, x = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    u = ((x + 0.5) / W).astype(np.float32).ravel()
    v = ((y + 0.5) / H).astype(np.float32).ravel()
    out = []
    for t in ts:
        out.append(np.stack([u, v, np.full_like(u, np.float32(t))], axis=1))
    return np.concatenate(out, axis=0)


def uniform_queries(n: int, g: np.random.Generator) -> np.ndarray:
    """n queries with u, v, t uniform in [0, 1): [n][3] float32."""
    q = g.random(size=(n, 3), dtype=np.float32)
    return np.minimum(q, np.float32(np.nextafter(np.float32(1), np.float32(0))))


# ------------------------------------------------------------------ virtual texturing

def vt_map_sides(n_maps: int, g: np.random.Generator, page: int = 128) -> np.ndarray:
    """Square map sides 128 * round(2^U[1, 5]) in [256, 4096]."""
    return page * np.round(2.0 ** g.uniform(1.0, 5.0, size=n_maps)).astype(np.int64)


def vt_requests(sides, n_req: int, g: np.random.Generator, page: int = 128,
                zipf_s: float = 1.1):
    """Page requests of one frame: arrays (model, page_x, page_y, t).

    The map of each request is drawn Zipf(s) over a random ranking of the maps, the page
    uniformly inside that map and t uniformly in [0, 1).
    """
    n_maps = len(sides)
    rank = g.permutation(n_maps)
    p = 1.0 / np.arange(1, n_maps + 1) ** zipf_s
    p /= p.sum()
    which = rank[g.choice(n_maps, size=n_req, p=p)]
    npg = np.asarray(sides)[which] // page
    px = (g.random(n_req) * npg).astype(np.int64)
    py = (g.random(n_req) * npg).astype(np.int64)
    t = g.random(n_req, dtype=np.float32)
    return which.astype(np.int32), px.astype(np.int32), py.astype(np.int32), t


# ------------------------------------------------------------- synthetic lightmap target

def light_scene(W: int, H: int, g: np.random.Generator, n_lights: int = 64,
                n_rects: int = 200) -> dict:
    """Parameters of the synthetic temporal lightmap (lights and moving occluders)."""
    s = W / 1024.0
    return dict(
        W=W, H=H,
        mu=np.stack([g.uniform(0, W, n_lights), g.uniform(0, H, n_lights)], 1),
        sigma=g.uniform(8.0, 64.0, n_lights) * s,
        amp=10.0 ** g.uniform(-1.0, 1.0, n_lights),
        colour=g.uniform(0.5, 1.0, (n_lights, 3)),
        phase=g.uniform(0.0, 1.0, n_lights),
        rc=np.stack([g.uniform(0, W, n_rects), g.uniform(0, H, n_rects)], 1),
        rhalf=g.uniform(4.0, 32.0, (n_rects, 2)) * s,
        rrad=g.uniform(0.0, 32.0, n_rects) * s,
        rphase=g.uniform(0.0, 1.0, n_rects),
        ambient=1e-3,
    )


def scene_frame_torch(scene: dict, t: float, device="cpu", rows=None):
    """One frame of the target at time t, evaluated at texel centres: torch [H][W][3] f32.

    I = ambient + M * sum_l colour_l * amp_l * (1 + sin 2pi(t + phase_l))/2 *
    exp(-|p - mu_l|^2 / (2 sigma_l^2)), where M is 0 inside any occluder rectangle whose
    centre moves on a circle of radius rrad with period 1.  ``rows`` selects a row range.
    """
    import torch
    W, H = scene["W"], scene["H"]
    y_lo, y_hi = (0, H) if rows is None else rows
    f32 = dict(dtype=torch.float32, device=device)
    ys = torch.arange(y_lo, y_hi, **f32) + 0.5
    xs = torch.arange(W, **f32) + 0.5
    out = torch.zeros((y_hi - y_lo, W, 3), **f32)
    mu = torch.tensor(scene["mu"], **f32)
    sig = torch.tensor(scene["sigma"], **f32)
    a = torch.tensor(scene["amp"] * 0.5 * (1.0 + np.sin(2 * np.pi * (t + scene["phase"]))), **f32)
    col = torch.tensor(scene["colour"], **f32)
    for l in range(mu.shape[0]):
        gx = torch.exp(-((xs - mu[l, 0]) ** 2) / (2 * sig[l] ** 2))
        gy = torch.exp(-((ys - mu[l, 1]) ** 2) / (2 * sig[l] ** 2))
        out += (a[l] * gy[:, None] * gx[None, :])[..., None] * col[l]
    ang = 2 * np.pi * (t + scene["rphase"])
    cx = scene["rc"][:, 0] + scene["rrad"] * np.cos(ang)
    cy = scene["rc"][:, 1] + scene["rrad"] * np.sin(ang)
    lit = torch.ones((y_hi - y_lo, W), dtype=torch.bool, device=device)
    for r in range(cx.shape[0]):
        inx = (xs - float(cx[r])).abs() <= float(scene["rhalf"][r, 0])
        iny = (ys - float(cy[r])).abs() <= float(scene["rhalf"][r, 1])
        lit &= ~(iny[:, None] & inx[None, :])
    return scene["ambient"] + out * lit[..., None].to(torch.float32)


def scene_target_torch(scene: dict, T: int, device="cpu"):
    """Full target [T][H][W][3] float16 (round to nearest even), frames at t_k = k/T."""
    import torch
    W, H = scene["W"], scene["H"]
    out = torch.empty((T, H, W, 3), dtype=torch.float16, device=device)
    step = max(1, (1 << 22) // W)
    for k in range(T):
        for y0 in range(0, H, step):
            y1 = min(H, y0 + step)
            out[k, y0:y1] = scene_frame_torch(scene, k / T, device, (y0, y1)).to(torch.float16)
    return out


# ------------------------------------------------------------------------ training

def train_samples(B: int, W: int, H: int, T: int, g: np.random.Generator):
    """B training samples (x, y, k) drawn uniformly with replacement."""
    x = g.integers(0, W, size=B)
    y = g.integers(0, H, size=B)
    k = g.integers(0, T, size=B)
    return x.astype(np.int64), y.astype(np.int64), k.astype(np.int64)


def pack_samples(x, y, k) -> np.ndarray:
    """Packed uint32 sample words x | y << 12 | k << 24 (x, y < 4096, k < 256)."""
    x = np.asarray(x, dtype=np.uint32)
    y = np.asarray(y, dtype=np.uint32)
    k = np.asarray(k, dtype=np.uint32)
    assert x.max(initial=0) < 4096 and y.max(initial=0) < 4096 and k.max(initial=0) < 256
    return x | (y << np.uint32(12)) | (k << np.uint32(24))


def train_init(W: int, H: int, Gw: int, Gh: int, T: int, mean_rgb, g: np.random.Generator) -> dict:
    """Initial trainable state (float32).

    e1 ~ U[0, 0.5), e2 ~ U[0.5, 1], w ~ U[0, 1], grid ~ N(0, 0.1^2), decoder He-normal
    with zero biases except b3 = log(mean target per channel).
    """
    ep = np.stack([g.uniform(0.0, 0.5, (H // 4, W // 4, N_CH)),
                   g.uniform(0.5, 1.0, (H // 4, W // 4, N_CH))], axis=-1).astype(np.float32)
    w = g.uniform(0.0, 1.0, (H, W, N_CH)).astype(np.float32)
    grid = (0.1 * g.standard_normal((T, Gh, Gw, N_CH))).astype(np.float32)
    mlp = he_normal_mlp(np.float32, g)
    mlp[MLP_SIZE - 3:] = np.log(np.maximum(np.asarray(mean_rgb, dtype=np.float64), 1e-6)).astype(np.float32)
    return dict(dims=dict(W=W, H=H, Gw=Gw, Gh=Gh, T=T), endpoints=ep, weights=w, grid=grid, mlp=mlp)


# ---------------------------------------------------------- large inputs drawn on device

def random_model_torch(W: int, H: int, Gw: int, Gh: int, T: int, seed: int, device="cuda",
                       grid_dtype="float16", mlp_dtype="float16") -> dict:
    """Same distributions as :func:`random_model`, drawn with torch on ``device`` (for sizes
    where host generation and upload would dominate).  Returns torch tensors."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    bc4 = torch.randint(0, 256, (H // 4, W // 4, N_CH, 8), generator=gen, device=device, dtype=torch.uint8)
    grid = (torch.rand((T, Gh, Gw, N_CH), generator=gen, device=device) * 2.0 - 1.0).to(getattr(torch, grid_dtype))
    parts = []
    for (fo, fi) in ((HIDDEN, N_IN), (HIDDEN, HIDDEN), (N_OUT, HIDDEN)):
        parts.append(torch.randn(fo * fi, generator=gen, device=device) * math.sqrt(2.0 / fi))
        parts.append(torch.zeros(fo, device=device))
    mlp = torch.cat(parts).to(getattr(torch, mlp_dtype))
    return dict(W=W, H=H, Gw=Gw, Gh=Gh, T=T, bc4=bc4, grid=grid, mlp=mlp)


def uniform_queries_torch(n: int, seed: int, device="cuda"):
    """n queries with u, v, t uniform in [0, 1): torch [n][3] float32 on ``device``."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    return torch.rand((n, 3), generator=gen, device=device, dtype=torch.float32)


def train_init_torch(W: int, H: int, Gw: int, Gh: int, T: int, mean_rgb, seed: int,
                     device="cuda") -> dict:
    """Same distributions as :func:`train_init`, drawn with torch on ``device`` as one flat
    float32 tensor in the trainer's layout (for sizes where host generation and upload would
    dominate).  The decoder is drawn on the host by :func:`he_normal_mlp`."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    f32 = dict(dtype=torch.float32, device=device)
    nb = (H // 4) * (W // 4) * N_CH
    ep = torch.empty((nb, 2), **f32)
    ep[:, 0].uniform_(0.0, 0.5, generator=gen)
    ep[:, 1].uniform_(0.5, 1.0, generator=gen)
    w = torch.empty(H * W * N_CH, **f32).uniform_(0.0, 1.0, generator=gen)
    grid = torch.empty(T * Gh * Gw * N_CH, **f32).normal_(0.0, 0.1, generator=gen)
    mlp = he_normal_mlp(np.float32, rng(seed, P_INIT))
    mlp[MLP_SIZE - 3:] = np.log(np.maximum(np.asarray(mean_rgb, dtype=np.float64), 1e-6)).astype(np.float32)
    flat = torch.cat([ep.reshape(-1), w, grid, torch.from_numpy(mlp).to(device)])
    return dict(dims=dict(W=W, H=H, Gw=Gw, Gh=Gh, T=T), flat=flat)


def train_samples_torch(B: int, W: int, H: int, T: int, seed: int, device="cuda", border: int = 0):
    """Packed samples (x | y << 12 | k << 24) drawn uniformly with replacement, on device.
    With a border of b texels the positions are drawn over the map padded by b on each
    side and folded back into it by mirror addressing (-1 - i below 0, 2n - 1 - i from n),
    i.e. uniform samples of the mirror-padded target (b <= min(W, H))."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    x = torch.randint(0, W + 2 * border, (B,), generator=gen, device=device, dtype=torch.int32)
    y = torch.randint(0, H + 2 * border, (B,), generator=gen, device=device, dtype=torch.int32)
    k = torch.randint(0, T, (B,), generator=gen, device=device, dtype=torch.int32)
    if border:
        assert border <= min(W, H)
        x, y = x - border, y - border
        x = torch.where(x < 0, -1 - x, torch.where(x >= W, 2 * W - 1 - x, x))
        y = torch.where(y < 0, -1 - y, torch.where(y >= H, 2 * H - 1 - y, y))
    return x | (y << 12) | (k << 24)
