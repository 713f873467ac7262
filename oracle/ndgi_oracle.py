"""Plain CPU reference ("oracle") for the Neural Dynamic GI decode and training path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this package.
The product path (the HIP library and its Python binding) never imports it and
shares no code, tables or helpers with it.

Everything here is float64 numpy (integer numpy for the block-compression codec),
written to be checked by eye against the paper (arXiv 2604.12625):

* Sec. 3.1, Eq. (3): the lighting at (u, v, t) is the output of a model H_Theta.
* Sec. 3.3, Eq. (4)-(5): features are sampled from a spatial map and a
  spatio-temporal map, concatenated and fed to a small MLP decoder G_Phi.
* Sec. 3.4, Eq. (6)-(7) and supplementary Sec. B: a 4x4 block stores two
  endpoints and per-texel weights; each texel is the linear interpolation of the
  endpoints (block compression, BC).
* Sec. 4 (Implementation): Adam, L2 loss.
* Supplementary Sec. D.2: tiled PSNR with the dynamic range taken per tile.
* Tables 2-3: bits per pixel accounting.

Two feature layouts are covered: an 8-channel BC4 spatial map plus an 8-channel
FP16/FP32 grid at quarter resolution with a 16-32-32-3 ReLU decoder and exponential
output, and the paper's hybrid layout (F_uv, F_ut, F_vt, F_uvt and gamma(t) into a
16-h-h-3 GELU decoder, Sec. 3.3); each place where the paper
does not fix a detail carries a "Reading" note.  Parity of the end-to-end decode
is the composition of separately pinned parts (codec, interpolation, MLP); the
trained quality of a model has no published value to pin against
("parity unpinned" for trained PSNR).
"""
from __future__ import annotations

import numpy as np

N_SPATIAL = 8      # channels of the block-compressed spatial map
N_GRID = 8         # channels of the spatio-temporal grid
N_IN = N_SPATIAL + N_GRID
HIDDEN = 32
N_OUT = 3

# Offsets of the packed decoder parameters: [W1 32x16 | b1 | W2 32x32 | b2 | W3 3x32 | b3]
# (row-major W[out][in], y = W x + b).
MLP_W1 = 0
MLP_B1 = MLP_W1 + HIDDEN * N_IN
MLP_W2 = MLP_B1 + HIDDEN
MLP_B2 = MLP_W2 + HIDDEN * HIDDEN
MLP_W3 = MLP_B2 + HIDDEN
MLP_B3 = MLP_W3 + N_OUT * HIDDEN
MLP_SIZE = MLP_B3 + N_OUT  # 1699


# --------------------------------------------------------------------------------------
# Block compression (BC4: one channel, 4x4 texels, 8 bytes)
# --------------------------------------------------------------------------------------

def bc4_palette(e0: int, e1: int) -> list[int]:
    """The eight 8-bit values a BC4 block with endpoints (e0, e1) can select.

    Follows Eq. (7) / supplementary Eq. (5): value = (1 - w) e_a + w e_b with w on a
    uniform grid.  Reading: two modes as in the public BC4 format; with e0 > e1 the
    six interior codes use w = j/7 (j = 1..6), otherwise four interior codes use
    w = j/5 (j = 1..4) and the last two codes are the constants 0 and 255.  The
    rational value is rounded to the nearest integer (the denominators are odd, so no
    ties occur): floor((N + (D-1)/2) / D) for numerator N and denominator D.
    """
    e0 = int(e0)
    e1 = int(e1)
    pal = [e0, e1]
    if e0 > e1:
        for j in range(1, 7):
            pal.append(((7 - j) * e0 + j * e1 + 3) // 7)
    else:
        for j in range(1, 5):
            pal.append(((5 - j) * e0 + j * e1 + 2) // 5)
        pal += [0, 255]
    return pal


def bc4_codes(block: np.ndarray) -> np.ndarray:
    """3-bit selector of each of the 16 texels of one 8-byte block, texel s = 4*row + col.

    Bytes 2..7 form a little-endian 48-bit field; texel s uses bits 3s..3s+2.
    """
    field = 0
    for b in range(6):
        field |= int(block[2 + b]) << (8 * b)
    return np.array([(field >> (3 * s)) & 7 for s in range(16)], dtype=np.int64)


def bc4_decode_block(block: np.ndarray) -> np.ndarray:
    """Decode one 8-byte BC4 block to a 4x4 uint8 array [row][col]."""
    pal = bc4_palette(block[0], block[1])
    codes = bc4_codes(block)
    return np.array([pal[c] for c in codes], dtype=np.uint8).reshape(4, 4)


def bc4_palette_value(e0: np.ndarray, e1: np.ndarray, code: np.ndarray) -> np.ndarray:
    """Vectorised palette lookup (same definition as :func:`bc4_palette`)."""
    e0 = e0.astype(np.int64)
    e1 = e1.astype(np.int64)
    code = code.astype(np.int64)
    j = code - 1                                   # interior codes 2.. map to j = 1..
    v8 = ((7 - j) * e0 + j * e1 + 3) // 7
    v6 = ((5 - j) * e0 + j * e1 + 2) // 5
    v6 = np.where(code == 6, 0, np.where(code == 7, 255, v6))
    interior = np.where(e0 > e1, v8, v6)
    out = np.where(code == 0, e0, np.where(code == 1, e1, interior))
    return out.astype(np.uint8)


def bc4_decode_blocks(blocks: np.ndarray) -> np.ndarray:
    """Decode n blocks ([n][8] uint8) to [n][16] uint8 (texel s = 4*row + col)."""
    blocks = np.asarray(blocks, dtype=np.uint8).reshape(-1, 8)
    field = np.zeros(blocks.shape[0], dtype=np.int64)
    for b in range(6):
        field |= blocks[:, 2 + b].astype(np.int64) << (8 * b)
    s = np.arange(16, dtype=np.int64)
    codes = (field[:, None] >> (3 * s)[None, :]) & 7
    e0 = np.repeat(blocks[:, 0:1], 16, axis=1)
    e1 = np.repeat(blocks[:, 1:2], 16, axis=1)
    return bc4_palette_value(e0, e1, codes)


def spatial_texels(bc4: np.ndarray, xs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """uint8 values of the 8 spatial channels at integer texels (xs, ys) -> [..., 8].

    ``bc4`` is [H/4][W/4][8 channels][8 bytes]: the eight single-channel blocks of a
    4x4 footprint are stored next to each other.
    """
    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    blocks = bc4[ys >> 2, xs >> 2]                       # [..., 8, 8]
    field = np.zeros(blocks.shape[:-1], dtype=np.int64)   # [..., 8]
    for b in range(6):
        field |= blocks[..., 2 + b].astype(np.int64) << (8 * b)
    slot = (4 * (ys & 3) + (xs & 3))[..., None]
    codes = (field >> (3 * slot)) & 7
    return bc4_palette_value(blocks[..., 0], blocks[..., 1], codes)


# --------------------------------------------------------------------------------------
# Feature sampling (Sec. 3.3) and the decoder MLP
# --------------------------------------------------------------------------------------

def _axis(coord: np.ndarray, size: int):
    """Texel-centre linear interpolation along one axis with clamp-to-edge.

    Reading: a coordinate c in [0, 1) maps to the continuous texel position
    c*size - 0.5; the two neighbours are floor() and floor()+1, clamped to [0, size-1].
    Returns (index0, index1, weight0, weight1).
    """
    p = coord * size - 0.5
    p0 = np.floor(p)
    f = p - p0
    i0 = np.clip(p0.astype(np.int64), 0, size - 1)
    i1 = np.clip(p0.astype(np.int64) + 1, 0, size - 1)
    return i0, i1, 1.0 - f, f


def _time_keys(t: np.ndarray, T: int):
    """Keys and weights for linear interpolation in time.

    Reading: T uniformly spaced keys at t_k = k/T on a periodic day cycle; t is
    wrapped into [0, 1) and interpolation between the last key and key 0 wraps.
    """
    tw = t - np.floor(t)
    tau = tw * T
    k = np.floor(tau)
    ft = tau - k
    k0 = np.mod(k.astype(np.int64), T)
    k1 = np.mod(k0 + 1, T)
    return k0, k1, 1.0 - ft, ft


def features(model: dict, u: np.ndarray, v: np.ndarray, t: np.ndarray) -> np.ndarray:
    """The 16 decoder inputs at (u, v, t) in float64: [S_0..S_7, G_0..G_7].

    S: bilinear sample of the decoded spatial map (value/255, Eq. (6) puts features
    in [0, 1]).  G: bilinear in space and linear in time sample of the grid
    [T][Gh][Gw][8] (the spatio-temporal feature map sampled at (u, v, t), Sec. 3.3).
    """
    W, H = model["W"], model["H"]
    x0, x1, wx0, wx1 = _axis(u, W)
    y0, y1, wy0, wy1 = _axis(v, H)
    bc4 = model["bc4"]
    S = np.zeros(u.shape + (N_SPATIAL,), dtype=np.float64)
    for (yy, wy) in ((y0, wy0), (y1, wy1)):
        for (xx, wx) in ((x0, wx0), (x1, wx1)):
            tex = spatial_texels(bc4, xx, yy).astype(np.float64) / 255.0
            S += (wx * wy)[..., None] * tex

    Gw, Gh, T = model["Gw"], model["Gh"], model["T"]
    grid = np.asarray(model["grid"])                         # [T][Gh][Gw][8], as stored
    gx0, gx1, gwx0, gwx1 = _axis(u, Gw)
    gy0, gy1, gwy0, gwy1 = _axis(v, Gh)
    k0, k1, wt0, wt1 = _time_keys(t, T)
    G = np.zeros(u.shape + (N_GRID,), dtype=np.float64)
    for (kk, wt) in ((k0, wt0), (k1, wt1)):
        for (yy, wy) in ((gy0, gwy0), (gy1, gwy1)):
            for (xx, wx) in ((gx0, gwx0), (gx1, gwx1)):
                G += (wt * wy * wx)[..., None] * grid[kk, yy, xx].astype(np.float64)
    return np.concatenate([S, G], axis=-1)


def unpack_mlp(mlp) -> dict:
    """Split the packed 1699-vector into float64 W1, b1, W2, b2, W3, b3."""
    p = np.asarray(mlp).astype(np.float64).reshape(-1)
    assert p.size == MLP_SIZE
    return dict(
        W1=p[MLP_W1:MLP_B1].reshape(HIDDEN, N_IN), b1=p[MLP_B1:MLP_W2],
        W2=p[MLP_W2:MLP_B2].reshape(HIDDEN, HIDDEN), b2=p[MLP_B2:MLP_W3],
        W3=p[MLP_W3:MLP_B3].reshape(N_OUT, HIDDEN), b3=p[MLP_B3:MLP_SIZE],
    )


def mlp_forward(mlp, x: np.ndarray) -> np.ndarray:
    """Decoder G_Phi: two ReLU hidden layers of width 32, exponential output -> HDR RGB."""
    P = unpack_mlp(mlp)
    h1 = np.maximum(0.0, x @ P["W1"].T + P["b1"])
    h2 = np.maximum(0.0, h1 @ P["W2"].T + P["b2"])
    z = h2 @ P["W3"].T + P["b3"]
    return np.exp(z)


def decode_f64(model: dict, u: np.ndarray, v: np.ndarray, t: np.ndarray) -> np.ndarray:
    """I(u, v, t) = H_Theta(u, v, t) (Eq. (3)) with float64 coordinates -> [n][3]."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    finite = np.isfinite(u) & np.isfinite(v) & np.isfinite(t)
    uu = np.where(finite, u, 0.0)
    vv = np.where(finite, v, 0.0)
    tt = np.where(finite, t, 0.0)
    rgb = mlp_forward(model["mlp"], features(model, uu, vv, tt))
    # Reading: a query with a non-finite coordinate has no defined texel; it
    # decodes to NaN in every channel.
    return np.where(finite[..., None], rgb, np.nan)


def decode(model: dict, uvt: np.ndarray) -> np.ndarray:
    """Decode explicit queries; ``uvt`` is [n][3] float32 (converted exactly to float64)."""
    q = np.asarray(uvt, dtype=np.float32).astype(np.float64).reshape(-1, 3)
    return decode_f64(model, q[:, 0], q[:, 1], q[:, 2])


def page_texels(model: dict, page_x: int, page_y: int, page: int):
    """Texel coordinates (x, y) and exact float64 texel-centre (u, v) of one VT page."""
    j, i = np.meshgrid(np.arange(page), np.arange(page), indexing="ij")
    x = page * page_x + i
    y = page * page_y + j
    u = (x + 0.5) / model["W"]
    v = (y + 0.5) / model["H"]
    return x, y, u, v


def decode_page(model: dict, page_x: int, page_y: int, t: float, page: int = 128) -> np.ndarray:
    """Decode one virtual-texturing page (Sec. 3.5, supplementary Sec. C): [page][page][3]."""
    _, _, u, v = page_texels(model, page_x, page_y, page)
    tt = np.full(u.shape, np.float64(np.float32(t)))
    return decode_f64(model, u, v, tt)


def decode_pages(models: list, reqs: list, page: int, dst: np.ndarray, pitch: int) -> int:
    """Write each valid request's page into ``dst`` ([rows*pitch][3]); returns #invalid.

    A request is (model, page_x, page_y, t, dst_offset); texel (i, j) of the page goes to
    dst[dst_offset + j*pitch + i].  A request whose model index or page lies outside its
    map is skipped and counted.
    """
    bad = 0
    for (m, px, py, t, off) in reqs:
        if not (0 <= m < len(models)):
            bad += 1
            continue
        md = models[m]
        if px < 0 or py < 0 or page * (px + 1) > md["W"] or page * (py + 1) > md["H"]:
            bad += 1
            continue
        rgb = decode_page(md, px, py, t, page)
        for j in range(page):
            dst[off + j * pitch: off + j * pitch + page] = rgb[j]
    return bad


# --------------------------------------------------------------------------------------
# BC7 mode 6 (the single-subset RGBA mode): one interpolation weight per texel shared by 4
# channels, as Eq. (6)-(7) write it (w_p in [0, 1] per pixel, e1, e2 in [0, 1]^k)
# --------------------------------------------------------------------------------------
# A 16-byte block read as a 128-bit little-endian integer: bits 0..6 hold the mode (mode 6:
# bit 6 set, bits 0..5 clear); then 7-bit endpoint values R0 R1 G0 G1 B0 B1 A0 A1 (bits
# 7..62); p-bits P0 (bit 63) and P1 (bit 64); then the texel indices, texel 0 with 3 bits
# (65..67, its top bit implied 0) and texel i >= 1 with 4 bits at 64 + 4 i.  Endpoint k of
# channel c is the 8-bit value (v << 1) | P_k; texel value ((64 - w) E0 + w E1 + 32) >> 6
# with w from the format's 4-bit weight table.
BC7_WEIGHTS4 = (0, 4, 9, 13, 17, 21, 26, 30, 34, 38, 43, 47, 51, 55, 60, 64)


def bc7m6_fields(block):
    """(E0 [4], E1 [4], idx [16]) of one mode-6 block (bytes) as python ints."""
    b = int.from_bytes(bytes(np.asarray(block, dtype=np.uint8)), "little")
    assert b & 0x7F == 0x40, "not a mode 6 block"
    v = [(b >> (7 + 7 * k)) & 0x7F for k in range(8)]
    p0, p1 = (b >> 63) & 1, (b >> 64) & 1
    E0 = [(v[2 * c] << 1) | p0 for c in range(4)]
    E1 = [(v[2 * c + 1] << 1) | p1 for c in range(4)]
    idx = [(b >> 65) & 7] + [(b >> (64 + 4 * i)) & 0xF for i in range(1, 16)]
    return E0, E1, idx


def bc7m6_decode_block(block) -> np.ndarray:
    """[16 texels][4 channels] uint8 of one mode-6 block (texel s = 4 * row + col)."""
    E0, E1, idx = bc7m6_fields(block)
    out = np.zeros((16, 4), dtype=np.uint8)
    for s_ in range(16):
        w = BC7_WEIGHTS4[idx[s_]]
        for c in range(4):
            out[s_, c] = ((64 - w) * E0[c] + w * E1[c] + 32) >> 6
    return out


def _bc7_take(B, pos, n):
    """Bits pos .. pos + n - 1 (n <= 8) of each block of B [..., 17] (bytes, int64, padded)."""
    pos = np.broadcast_to(np.asarray(pos, dtype=np.int64), B.shape[:-1])
    byte = (pos >> 3)[..., None]
    lo = np.take_along_axis(B, byte, -1)[..., 0]
    hi = np.take_along_axis(B, np.minimum(byte + 1, 16), -1)[..., 0]
    return ((lo | (hi << 8)) >> (pos & 7)) & ((1 << n) - 1)


def bc7_texels(blocks: np.ndarray, xs, ys) -> np.ndarray:
    """Vectorised decode of texels (xs, ys) from their selected 16-byte blocks [..., 16] -> [..., 4]
    (modes 4, 5 and 6; zeros for other modes), as bc7_decode_block."""
    blocks = np.asarray(blocks, dtype=np.uint8)
    B = np.concatenate([blocks, np.zeros(blocks.shape[:-1] + (1,), np.uint8)], axis=-1).astype(np.int64)
    slot = (4 * (np.asarray(ys) & 3) + (np.asarray(xs) & 3)).astype(np.int64)
    slot = np.broadcast_to(slot, B.shape[:-1])
    b0 = B[..., 0]
    mode = np.where(b0 & 0x10, 4, np.where(b0 & 0x20, 5, np.where(b0 & 0x40, 6, -1)))
    mode = np.where(b0 & 0x0F, -1, mode)     # modes 0-3 (and 7 / reserved below) decode to 0

    def idx(P, bits):     # the texel's index in a set starting at bit P
        pos = np.where(slot == 0, P, P + bits - 1 + bits * (slot - 1))
        return np.where(slot == 0, _bc7_take(B, pos, bits - 1), _bc7_take(B, pos, bits))

    def expand(v, n):
        return (v << (8 - n)) | (v >> (2 * n - 8)) if n < 8 else v

    def lerp(e0, e1, w):
        return ((64 - w) * e0 + w * e1 + 32) >> 6
    W2, W3, W4 = (np.asarray(BC7_WEIGHTS[k], dtype=np.int64) for k in (2, 3, 4))
    out = np.zeros(B.shape[:-1] + (4,), dtype=np.int64)
    # mode 6
    p0, p1 = _bc7_take(B, 63, 1), _bc7_take(B, 64, 1)
    w6 = W4[idx(65, 4)]
    m6 = np.stack([lerp((_bc7_take(B, 7 + 14 * c, 7) << 1) | p0, (_bc7_take(B, 14 + 14 * c, 7) << 1) | p1, w6)
                   for c in range(4)], axis=-1)
    # mode 5
    wc5, wa5 = W2[idx(66, 2)], W2[idx(97, 2)]
    m5 = np.stack([lerp(expand(_bc7_take(B, 8 + 14 * c, 7), 7), expand(_bc7_take(B, 15 + 14 * c, 7), 7), wc5)
                   for c in range(3)] + [lerp(_bc7_take(B, 50, 8), _bc7_take(B, 58, 8), wa5)], axis=-1)
    # mode 4
    sel = _bc7_take(B, 7, 1)
    w2, w3 = W2[idx(50, 2)], W3[idx(81, 3)]
    wc4, wa4 = np.where(sel == 1, w3, w2), np.where(sel == 1, w2, w3)
    m4 = np.stack([lerp(expand(_bc7_take(B, 8 + 10 * c, 5), 5), expand(_bc7_take(B, 13 + 10 * c, 5), 5), wc4)
                   for c in range(3)] + [lerp(expand(_bc7_take(B, 38, 6), 6), expand(_bc7_take(B, 44, 6), 6), wa4)],
                  axis=-1)
    for m, val, rpos in ((4, m4, 5), (5, m5, 6)):
        rot = _bc7_take(B, rpos, 2)
        for r in (1, 2, 3):
            sw = (rot == r)[..., None]
            v2 = val.copy()
            v2[..., r - 1], v2[..., 3] = val[..., 3], val[..., r - 1]
            val = np.where(sw, v2, val)
        out = np.where((mode == m)[..., None], val, out)
    out = np.where((mode == 6)[..., None], m6, out)
    return out.astype(np.uint8)


# --------------------------------------------------------------------------------------
# BC7 modes 4, 5 and 6: the format's single-subset modes that carry four channels.  Modes 4
# and 5 hold the colour (R, G, B) and alpha endpoints apart, each with its own index set,
# and a 2-bit rotation swaps alpha with one colour channel after decoding (1: R, 2: G, 3:
# B); mode 4 has 5-bit colour and 6-bit alpha endpoints, 2-bit and 3-bit indices (its index
# selection bit gives the 3-bit set to colour when 1), mode 5 7-bit colour and 8-bit alpha
# endpoints and 2-bit indices for both.  Fields in bit order from bit 0: the mode (m zero
# bits then a one), then mode 4: rotation (2), selection (1), R0 R1 G0 G1 B0 B1 (5 each),
# A0 A1 (6 each), the 2-bit index set (31 bits), the 3-bit set (47 bits); mode 5: rotation
# (2), R0 .. B1 (7 each), A0 A1 (8 each), colour indices (31), alpha indices (31); mode 6
# as above.  In every index set texel 0 drops its top bit (it is 0).  An n-bit endpoint
# value v is the 8-bit (v << (8 - n)) | (v >> (2n - 8)); a texel is
# ((64 - w) E0 + w E1 + 32) >> 6 with w from the b-bit weight table (64 j + (2^b - 1) / 2)
# / (2^b - 1).  Reading: blocks of modes 0-3 and 7 (partitioned or RGB only) and the
# reserved mode are not used by these feature maps and decode to zero texels.
BC7_WEIGHTS = {2: (0, 21, 43, 64), 3: (0, 9, 18, 27, 37, 46, 55, 64), 4: BC7_WEIGHTS4}


def bc7_mode(block) -> int:
    """Mode of a 16-byte block (the number of zero bits before the first one), 8 if none."""
    b0 = int(np.asarray(block, dtype=np.uint8)[0])
    for m in range(8):
        if (b0 >> m) & 1:
            return m
    return 8


def _bc7_expand(v: int, n: int) -> int:
    return ((v << (8 - n)) | (v >> (2 * n - 8))) if n < 8 else v


def bc7_fields(block):
    """(mode, rotation, E0 [4], E1 [4], colour indices [16], colour index bits, alpha indices
    [16], alpha index bits) of a mode 4, 5 or 6 block, endpoints as 8-bit values in
    R, G, B, A order before the rotation; None for any other mode."""
    b = int.from_bytes(bytes(np.asarray(block, dtype=np.uint8)), "little")
    m = bc7_mode(block)

    def take(pos, n):
        return (b >> pos) & ((1 << n) - 1)

    def index_set(pos, bits):
        out = [take(pos, bits - 1)]
        pos += bits - 1
        for _ in range(15):
            out.append(take(pos, bits))
            pos += bits
        return out
    if m == 6:
        E0, E1, idx = bc7m6_fields(block)
        return 6, 0, E0, E1, idx, 4, idx, 4
    if m == 5:
        rot = take(6, 2)
        col = [take(8 + 7 * k, 7) for k in range(6)]
        a0, a1 = take(50, 8), take(58, 8)
        E0 = [_bc7_expand(col[2 * c], 7) for c in range(3)] + [a0]
        E1 = [_bc7_expand(col[2 * c + 1], 7) for c in range(3)] + [a1]
        return 5, rot, E0, E1, index_set(66, 2), 2, index_set(97, 2), 2
    if m == 4:
        rot, sel = take(5, 2), take(7, 1)
        col = [take(8 + 5 * k, 5) for k in range(6)]
        a0, a1 = _bc7_expand(take(38, 6), 6), _bc7_expand(take(44, 6), 6)
        E0 = [_bc7_expand(col[2 * c], 5) for c in range(3)] + [a0]
        E1 = [_bc7_expand(col[2 * c + 1], 5) for c in range(3)] + [a1]
        i2, i3 = index_set(50, 2), index_set(81, 3)
        return (4, rot, E0, E1, i3, 3, i2, 2) if sel else (4, rot, E0, E1, i2, 2, i3, 3)
    return None


def bc7_decode_block(block) -> np.ndarray:
    """[16 texels][4 channels] uint8 of one BC7 block of mode 4, 5 or 6 (zeros otherwise)."""
    f = bc7_fields(block)
    out = np.zeros((16, 4), dtype=np.uint8)
    if f is None:
        return out
    _, rot, E0, E1, ci, cb, ai, ab = f
    for s_ in range(16):
        wc, wa = BC7_WEIGHTS[cb][ci[s_]], BC7_WEIGHTS[ab][ai[s_]]
        v = [((64 - wc) * E0[c] + wc * E1[c] + 32) >> 6 for c in range(3)]
        v.append(((64 - wa) * E0[3] + wa * E1[3] + 32) >> 6)
        if rot:
            v[rot - 1], v[3] = v[3], v[rot - 1]
        out[s_] = v
    return out


def bc7_quantise_endpoint(e4):
    """Mode-6 endpoint of 4 channel values in [0, 1] (last axis): the p-bit and 7-bit values
    whose 8-bit values (v << 1) | p are nearest to x = fl32(255 e) in summed squared error
    (v = rint((x - p) / 2) clamped to 0..127; ties keep p = 0).  Returns (E [..., 4], v7, p)."""
    x = (np.float32(255.0) * np.asarray(e4, dtype=np.float32)).astype(np.float64)
    cand = []
    for p in (0, 1):
        v7 = np.clip(np.rint((x - p) / 2.0), 0, 127).astype(np.int64)
        E = 2 * v7 + p
        cand.append((E, v7, ((E - x) ** 2).sum(-1)))
    take1 = cand[1][2] < cand[0][2]
    E = np.where(take1[..., None], cand[1][0], cand[0][0])
    v7 = np.where(take1[..., None], cand[1][1], cand[0][1])
    return E, v7, take1.astype(np.int64)


def quantise_weight4(w):
    """4-bit BC7 index J = round-half-even(fl32(15 * w))."""
    return np.rint(np.float32(15.0) * np.asarray(w, dtype=np.float32)).astype(np.int64)


def export_bc7(endpoints: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """Encode a BC7-simulated 4-channel map ([Hb][Wb][4][2] endpoints, [H][W] weights) as mode-6
    blocks [Hb][Wb][16].  Reading (the decode equals the simulation bit for bit): endpoints
    quantised by bc7_quantise_endpoint, index J = quantise_weight4(w); when texel 0's index
    has its top bit set the endpoints swap and every index becomes 15 - J (the weight table is
    symmetric, w(15 - J) = 64 - w(J))."""
    Hb, Wb = endpoints.shape[0], endpoints.shape[1]
    E0, v0, p0 = bc7_quantise_endpoint(endpoints[..., 0])
    E1, v1, p1 = bc7_quantise_endpoint(endpoints[..., 1])
    J = quantise_weight4(weights)
    out = np.zeros((Hb, Wb, 16), dtype=np.uint8)
    for by in range(Hb):
        for bx in range(Wb):
            a, b, pa, pb = v0[by, bx], v1[by, bx], int(p0[by, bx]), int(p1[by, bx])
            idx = [int(J[4 * by + s_ // 4, 4 * bx + s_ % 4]) for s_ in range(16)]
            if idx[0] >= 8:
                a, b, pa, pb = b, a, pb, pa
                idx = [15 - j for j in idx]
            bits = 0x40
            for c in range(4):
                bits |= int(a[c]) << (7 + 14 * c)
                bits |= int(b[c]) << (14 + 14 * c)
            bits |= pa << 63
            bits |= pb << 64
            bits |= idx[0] << 65
            for i in range(1, 16):
                bits |= idx[i] << (64 + 4 * i)
            out[by, bx] = np.frombuffer(bits.to_bytes(16, "little"), dtype=np.uint8)
    return out


# --------------------------------------------------------------------------------------
# Hybrid feature maps and the GELU decoder (Sec. 3.3, Eq. (4)-(5), Table 1, Table 3, Sec. 4)
# --------------------------------------------------------------------------------------
# A hybrid model holds four feature maps and a decoder:
#   fuv  [H/4][W/4][4][8]       F_uv, W x H x 4 channels, BC4 blocks (one per channel), or
#        [H/4][W/4][16]         with codec 1 one BC7 mode-6 block per footprint
#   fuvt [S][Gv/4][Gu/4][4][8]  F_uvt, Gu x Gv x 4 channels in S time slices, each slice
#                               block-compressed on its own (Sec. 3.4); [..][16] for codec 1
#   fut  [Tt][U][2]             F_ut, 8-bit, U x Tt x 2 channels
#   fvt  [Tt][V][2]             F_vt, 8-bit, V x Tt x 2 channels
#   keys [n]                    times of the baked lightmaps (n = 0: uniform time)
#   mlp                         packed [W1 h x 16 | b1 | W2 h x h | b2 | W3 3 x h | b3]
# Readings (the paper gives the structure, not these details):
# * every stored byte q stands for the feature value q / 255 (Eq. (6) puts features in
#   [0, 1]; the 8-bit planes use the same scale);
# * space: texel-centre bilinear with clamp-to-edge on every spatial axis, as for the
#   other layout;
# * time: t is clamped to [0, 1] (a day is not wrapped: the feature maps' time axes are
#   learned over one interval); the lightmaps' key times (Sec. 3.1: possibly non-uniform)
#   map t piecewise linearly to tau in [0, 1], key i going to i / (n - 1); the time axes
#   of F_ut, F_vt and F_uvt hold their samples at tau = k / (N - 1) (their ends at the
#   first and last key) and are interpolated linearly;
# * gamma(t) takes the clamped t itself (Eq. (4));
# * decoder inputs in the order of Eq. (4): [V_uvt (4), V_uv (4), V_ut (2), V_vt (2),
#   gamma (4)]; hidden layers use the exact GELU x * Phi(x) (Sec. 4; the erf form is the
#   PyTorch default), the output layer has no activation.
HYB_IN = 16


def hybrid_mlp_size(hidden: int) -> int:
    return hidden * HYB_IN + hidden + hidden * hidden + hidden + N_OUT * hidden + N_OUT


def unpack_hybrid_mlp(mlp, hidden: int) -> dict:
    p = np.asarray(mlp).astype(np.float64).reshape(-1)
    assert p.size == hybrid_mlp_size(hidden)
    o1 = hidden * HYB_IN
    o2 = o1 + hidden
    o3 = o2 + hidden * hidden
    o4 = o3 + hidden
    o5 = o4 + N_OUT * hidden
    return dict(W1=p[:o1].reshape(hidden, HYB_IN), b1=p[o1:o2], W2=p[o2:o3].reshape(hidden, hidden),
                b2=p[o3:o4], W3=p[o4:o5].reshape(N_OUT, hidden), b3=p[o5:])


def gelu(x: np.ndarray) -> np.ndarray:
    """GELU(x) = x Phi(x), Phi the standard normal CDF = (1 + erf(x / sqrt 2)) / 2."""
    from scipy.special import erf
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def hybrid_mlp_forward(mlp, hidden: int, x: np.ndarray) -> np.ndarray:
    """Decoder G_Phi of Eq. (4): two GELU hidden layers of width ``hidden``, linear output."""
    P = unpack_hybrid_mlp(mlp, hidden)
    h1 = gelu(x @ P["W1"].T + P["b1"])
    h2 = gelu(h1 @ P["W2"].T + P["b2"])
    return h2 @ P["W3"].T + P["b3"]


def gamma_t(t: np.ndarray) -> np.ndarray:
    """Positional encoding of time, Eq. (4): [sin(pi t), cos(pi t), sin(2 pi t), cos(2 pi t)]."""
    t = np.asarray(t, dtype=np.float64)
    return np.stack([np.sin(np.pi * t), np.cos(np.pi * t), np.sin(2 * np.pi * t), np.cos(2 * np.pi * t)], -1)


def key_time_coord(t: np.ndarray, keys) -> np.ndarray:
    """tau in [0, 1] for a clamped time t: piecewise linear through (keys[i], i / (n - 1));
    t = tau with no key table."""
    t = np.asarray(t, dtype=np.float64)
    k = np.asarray(keys, dtype=np.float64).reshape(-1)
    if k.size == 0:
        return t
    n = k.size
    i = np.clip(np.searchsorted(k, t, side="right") - 1, 0, n - 2)
    f = (t - k[i]) / (k[i + 1] - k[i])
    return np.clip((i + f) / (n - 1), 0.0, 1.0)


def _node_axis(tau: np.ndarray, N: int):
    """Linear interpolation over N samples at tau = k / (N - 1): (i0, i1, w0, w1)."""
    if N == 1:
        z = np.zeros(np.shape(tau), dtype=np.int64)
        return z, z, np.ones(np.shape(tau)), np.zeros(np.shape(tau))
    p = tau * (N - 1)
    i0 = np.minimum(np.floor(p).astype(np.int64), N - 2)
    f = p - i0
    return i0, i0 + 1, 1.0 - f, f


def bc4_texels(blocks: np.ndarray, xs, ys) -> np.ndarray:
    """Values of all channels of block-compressed texels (xs, ys): ``blocks`` is the
    [..., C, 8] selection of the texels' footprints; returns [..., C] uint8."""
    field = np.zeros(blocks.shape[:-1], dtype=np.int64)
    for b in range(6):
        field |= blocks[..., 2 + b].astype(np.int64) << (8 * b)
    slot = (4 * (np.asarray(ys) & 3) + (np.asarray(xs) & 3))[..., None]
    codes = (field >> (3 * slot)) & 7
    return bc4_palette_value(blocks[..., 0], blocks[..., 1], codes)


def _hyb_tex(model: dict, blocks, xs, ys) -> np.ndarray:
    """4-channel texel values / 255 of the selected footprints: BC4 per channel ([..., 4, 8]
    bytes, codec 0) or BC7 mode 6 ([..., 16] bytes, codec 1)."""
    if model.get("codec", 0) == 1:
        return bc7_texels(blocks, xs, ys) / 255.0
    return bc4_texels(blocks, xs, ys) / 255.0


def hybrid_features(model: dict, u: np.ndarray, v: np.ndarray, t: np.ndarray) -> np.ndarray:
    """The 16 decoder inputs at (u, v, t) (Eq. (4)), float64 -> [..., 16]."""
    tc = np.clip(t, 0.0, 1.0)
    tau = key_time_coord(tc, model["keys"])
    # V_uvt: bilinear in each of the two slices around tau, then linear between them
    Gu, Gv, S = model["Gu"], model["Gv"], model["S"]
    x0, x1, wx0, wx1 = _axis(u, Gu)
    y0, y1, wy0, wy1 = _axis(v, Gv)
    s0, s1, ws0, ws1 = _node_axis(tau, S)
    fuvt = model["fuvt"]
    Vuvt = np.zeros(np.shape(u) + (4,))
    for (ss, ws) in ((s0, ws0), (s1, ws1)):
        for (yy, wy) in ((y0, wy0), (y1, wy1)):
            for (xx, wx) in ((x0, wx0), (x1, wx1)):
                tex = _hyb_tex(model, fuvt[ss, yy >> 2, xx >> 2], xx, yy)
                Vuvt += (ws * wy * wx)[..., None] * tex
    # V_uv: bilinear in the W x H map
    x0, x1, wx0, wx1 = _axis(u, model["W"])
    y0, y1, wy0, wy1 = _axis(v, model["H"])
    fuv = model["fuv"]
    Vuv = np.zeros(np.shape(u) + (4,))
    for (yy, wy) in ((y0, wy0), (y1, wy1)):
        for (xx, wx) in ((x0, wx0), (x1, wx1)):
            Vuv += (wy * wx)[..., None] * _hyb_tex(model, fuv[yy >> 2, xx >> 2], xx, yy)
    # V_ut, V_vt: bilinear on the (u, t) and (v, t) planes
    k0, k1, wk0, wk1 = _node_axis(tau, model["Tt"])
    planes = []
    for (c, size, plane) in ((u, model["U"], model["fut"]), (v, model["V"], model["fvt"])):
        a0, a1, wa0, wa1 = _axis(c, size)
        P = np.zeros(np.shape(u) + (2,))
        for (kk, wk) in ((k0, wk0), (k1, wk1)):
            for (aa, wa) in ((a0, wa0), (a1, wa1)):
                P += (wk * wa)[..., None] * (plane[kk, aa].astype(np.float64) / 255.0)
        planes.append(P)
    return np.concatenate([Vuvt, Vuv, planes[0], planes[1], gamma_t(tc)], axis=-1)


def hybrid_decode_f64(model: dict, u, v, t) -> np.ndarray:
    """I(u, v, t) = G_Phi(V_uvt, V_uv, V_ut, V_vt, gamma(t)) (Eq. (4)) -> [n][3]; a query
    with a non-finite coordinate decodes to NaN."""
    u = np.asarray(u, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    finite = np.isfinite(u) & np.isfinite(v) & np.isfinite(t)
    x = hybrid_features(model, np.where(finite, u, 0.0), np.where(finite, v, 0.0), np.where(finite, t, 0.0))
    rgb = hybrid_mlp_forward(model["mlp"], model["hidden"], x)
    return np.where(finite[..., None], rgb, np.nan)


def hybrid_decode(model: dict, uvt: np.ndarray) -> np.ndarray:
    """Decode explicit float32 queries [n][3] of a hybrid model."""
    q = np.asarray(uvt, dtype=np.float32).astype(np.float64).reshape(-1, 3)
    return hybrid_decode_f64(model, q[:, 0], q[:, 1], q[:, 2])


def mirror_texel(i, n: int):
    """Mirror addressing of texel indices on a map of n texels (the graphics MIRROR mode:
    the map reflected about its edges, so texel -1 - k is texel k and texel n + k is texel
    n - 1 - k); one reflection, for indices in [-n, 2n)."""
    i = np.asarray(i)
    return np.where(i < 0, -1 - i, np.where(i >= n, 2 * n - 1 - i, i))


def hybrid_decode_pages(models: list, reqs: list, page: int, dst: np.ndarray, pitch: int, border: int = 0) -> int:
    """Page decode of hybrid models (same request convention as :func:`decode_pages`).

    With a border of b texels (supplementary Virtual Texturing section: tiles stored with a
    small border for hardware filtering, padded by mirroring) a request writes a (page + 2b)^2 region: its texel
    (i, j) is the decode at the texel centre of map texel (mirror_texel(page px - b + i, W),
    mirror_texel(page py - b + j, H)).  Inside the map the border holds the neighbouring
    texels; past the map's edge it mirrors the map (for a per-tile model, the tile)."""
    bad = 0
    R = page + 2 * border
    for (m, px, py, t, off) in reqs:
        if not (0 <= m < len(models)):
            bad += 1
            continue
        md = models[m]
        if px < 0 or py < 0 or page * (px + 1) > md["W"] or page * (py + 1) > md["H"]:
            bad += 1
            continue
        jj, ii = np.meshgrid(np.arange(R), np.arange(R), indexing="ij")
        x = mirror_texel(page * px - border + ii, md["W"])
        y = mirror_texel(page * py - border + jj, md["H"])
        u = (x + 0.5) / md["W"]
        v = (y + 0.5) / md["H"]
        rgb = hybrid_decode_f64(md, u, v, np.full(u.shape, np.float64(np.float32(t))))
        for j in range(R):
            dst[off + j * pitch: off + j * pitch + R] = rgb[j]
    return bad


# --------------------------------------------------------------------------------------
# Training with BC simulation (Sec. 3.4, Eq. (6)-(7); Sec. 4)
# --------------------------------------------------------------------------------------
# Trainable state (float32 master copies):
#   endpoints [H/4][W/4][8][2]  -- e1, e2 of each 4x4 block and channel, in [0, 1]
#   weights   [H][W][8]         -- per-texel interpolation weight w_p, in [0, 1]
#   grid      [T][Gh][Gw][8]
#   mlp       [1699]

def quantise_endpoint(e: np.ndarray) -> np.ndarray:
    """8-bit endpoint E = round-half-even(fl32(255 * e)) (float32 product, as stored)."""
    return np.rint(np.float32(255.0) * np.asarray(e, dtype=np.float32)).astype(np.int64)


def quantise_weight(w: np.ndarray) -> np.ndarray:
    """3-bit weight index J = round-half-even(fl32(7 * w))."""
    return np.rint(np.float32(7.0) * np.asarray(w, dtype=np.float32)).astype(np.int64)


def bcsim_value(E1: np.ndarray, E2: np.ndarray, J: np.ndarray) -> np.ndarray:
    """Eq. (7) at the quantised point w = J/7, rounded to the nearest 8-bit value."""
    return ((7 - J) * E1 + J * E2 + 3) // 7


def bcsim_spatial(endpoints: np.ndarray, weights: np.ndarray, xs, ys):
    """Spatial features of texels (xs, ys) under BC simulation.

    Returns (value_u8 [..,8], E1, E2, J) so the caller can form the straight-through
    derivatives.
    """
    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    ep = endpoints[ys >> 2, xs >> 2]          # [..., 8, 2]
    E1 = quantise_endpoint(ep[..., 0])
    E2 = quantise_endpoint(ep[..., 1])
    J = quantise_weight(weights[ys, xs])      # [..., 8]
    return bcsim_value(E1, E2, J), E1, E2, J


def _sample_coords(dims: dict, xs, ys):
    """Grid corners and weights of texel centres (xs, ys): same rule as :func:`_axis`."""
    W, H, Gw, Gh = dims["W"], dims["H"], dims["Gw"], dims["Gh"]
    u = (np.asarray(xs, dtype=np.float64) + 0.5) / W
    v = (np.asarray(ys, dtype=np.float64) + 0.5) / H
    gx0, gx1, wx0, wx1 = _axis(u, Gw)
    gy0, gy1, wy0, wy1 = _axis(v, Gh)
    return ((gy0, gx0, wy0 * wx0), (gy0, gx1, wy0 * wx1),
            (gy1, gx0, wy1 * wx0), (gy1, gx1, wy1 * wx1))


def train_forward(state: dict, xs, ys, ks, need_cache: bool = False):
    """Predicted HDR RGB at training samples (texel (x, y) of key k, i.e. t = k/T).

    Reading: samples sit exactly on a key, so the time weight of key k is 1 and the
    next key contributes 0; the spatial feature is the BC-simulated texel itself.
    """
    dims = state["dims"]
    val, E1, E2, J = bcsim_spatial(state["endpoints"], state["weights"], xs, ys)
    S = val.astype(np.float64) / 255.0
    grid = np.asarray(state["grid"])
    ks = np.asarray(ks, dtype=np.int64)
    corners = _sample_coords(dims, xs, ys)
    G = np.zeros(S.shape, dtype=np.float64)
    for (gy, gx, w) in corners:
        G += w[..., None] * grid[ks, gy, gx].astype(np.float64)
    x = np.concatenate([S, G], axis=-1)
    P = unpack_mlp(state["mlp"])
    a1 = x @ P["W1"].T + P["b1"]
    h1 = np.maximum(0.0, a1)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(0.0, a2)
    z = h2 @ P["W3"].T + P["b3"]
    rgb = np.exp(z)
    if not need_cache:
        return rgb
    cache = dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2, rgb=rgb, E1=E1, E2=E2, J=J,
                 corners=corners, P=P)
    return rgb, cache


def l2_loss(rgb: np.ndarray, target: np.ndarray) -> float:
    """L2 loss (Sec. 4): mean over samples and the three channels of (pred - target)^2."""
    d = rgb - np.asarray(target, dtype=np.float64)
    return float(np.sum(d * d) / d.size)


def train_grads(state: dict, xs, ys, ks, target: np.ndarray):
    """Loss and analytic gradients of every trainable array (same shapes as the state).

    Straight-through estimator (reading of "update the endpoints and weights",
    Sec. 3.4): the derivative is that of the unrounded Eq. (7),
    f = ((1 - w) e1 + w e2), evaluated at the quantised point e = E/255, w = J/7.
    ReLU'(0) is taken as 0.
    """
    dims = state["dims"]
    rgb, c = train_forward(state, xs, ys, ks, need_cache=True)
    target = np.asarray(target, dtype=np.float64)
    n = rgb.size
    loss = float(np.sum((rgb - target) ** 2) / n)
    P = c["P"]
    dz = (2.0 / n) * (rgb - target) * rgb                  # d/dz of exp output
    gW3 = dz.T @ c["h2"]
    gb3 = dz.sum(axis=0)
    dh2 = (dz @ P["W3"]) * (c["a2"] > 0)
    gW2 = dh2.T @ c["h1"]
    gb2 = dh2.sum(axis=0)
    dh1 = (dh2 @ P["W2"]) * (c["a1"] > 0)
    gW1 = dh1.T @ c["x"]
    gb1 = dh1.sum(axis=0)
    dx = dh1 @ P["W1"]
    dS = dx[:, :N_SPATIAL]                   # d loss / d f with f = value/255 in [0, 1]
    dG = dx[:, N_SPATIAL:]

    g_mlp = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])

    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    ks = np.asarray(ks, dtype=np.int64)
    J = c["J"].astype(np.float64)
    E1 = c["E1"].astype(np.float64)
    E2 = c["E2"].astype(np.float64)
    g_end = np.zeros(state["endpoints"].shape, dtype=np.float64)
    g_w = np.zeros(state["weights"].shape, dtype=np.float64)
    ch = np.arange(N_SPATIAL)
    bx = (xs >> 2)[:, None]
    by = (ys >> 2)[:, None]
    np.add.at(g_end, (by, bx, ch[None, :], 0), dS * (1.0 - J / 7.0))
    np.add.at(g_end, (by, bx, ch[None, :], 1), dS * (J / 7.0))
    np.add.at(g_w, (ys[:, None], xs[:, None], ch[None, :]), dS * (E2 - E1) / 255.0)

    g_grid = np.zeros(np.asarray(state["grid"]).shape, dtype=np.float64)
    for (gy, gx, w) in c["corners"]:
        np.add.at(g_grid, (ks[:, None], gy[:, None], gx[:, None], ch[None, :]),
                  w[:, None] * dG)
    return loss, dict(endpoints=g_end, weights=g_w, grid=g_grid, mlp=g_mlp)


def adam_update(param, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999,
                eps=1e-8):
    """One Adam step (Kingma & Ba; the bias-corrected form PyTorch uses), float64.

    ``step`` is the 1-based step count after this update.  Returns (param, m, v).
    """
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    bc1 = 1.0 - beta1 ** step
    bc2 = 1.0 - beta2 ** step
    denom = np.sqrt(v) / np.sqrt(bc2) + eps
    p = np.asarray(param, dtype=np.float64) - (lr / bc1) * m / denom
    return p, m, v


def train_step(state: dict, opt: dict, xs, ys, ks, target):
    """One full step: forward, L2 loss, backward, Adam on every array, projection.

    ``opt`` holds m/v arrays per key, 'step', 'lr_feat' (endpoints, weights, grid) and
    'lr_mlp'.  Reading: endpoints and weights are projected back to [0, 1] after the
    update (Eq. (6) constrains them to that interval).  Returns the loss.
    """
    loss, g = train_grads(state, xs, ys, ks, target)
    opt["step"] += 1
    for key in ("endpoints", "weights", "grid", "mlp"):
        lr = opt["lr_mlp"] if key == "mlp" else opt["lr_feat"]
        p, m, v = adam_update(state[key], g[key], opt["m"][key], opt["v"][key],
                              opt["step"], lr, opt.get("beta1", 0.9),
                              opt.get("beta2", 0.999), opt.get("eps", 1e-8))
        if key in ("endpoints", "weights"):
            p = np.clip(p, 0.0, 1.0)
        state[key] = p
        opt["m"][key] = m
        opt["v"][key] = v
    return loss


# --------------------------------------------------------------------------------------
# Export (Sec. 3.4 last paragraph): trained endpoints/weights -> real BC4 blocks
# --------------------------------------------------------------------------------------

def export_bc4(endpoints: np.ndarray, weights: np.ndarray) -> np.ndarray:
    """Encode a BC-simulated map as BC4 blocks [H/4][W/4][C][8] uint8 (C channels).

    Reading (one of several encodings that decode identically): with E1 > E2 the block
    is (e0, e1) = (E1, E2) in 8-value mode and weight J maps to code 0 (J = 0), 1 (J = 7)
    or J + 1; with E1 < E2 the endpoints swap and J becomes 7 - J; with E1 = E2 the block
    is (E, E) in 6-value mode with every code 0.
    """
    Hb, Wb, C = endpoints.shape[0], endpoints.shape[1], endpoints.shape[2]
    E1 = quantise_endpoint(endpoints[..., 0])        # [Hb][Wb][C]
    E2 = quantise_endpoint(endpoints[..., 1])
    J = quantise_weight(weights)                     # [H][W][C]
    out = np.zeros((Hb, Wb, C, 8), dtype=np.uint8)
    for by in range(Hb):
        for bx in range(Wb):
            for c in range(C):
                a, b = int(E1[by, bx, c]), int(E2[by, bx, c])
                field = 0
                for s in range(16):
                    j = int(J[4 * by + s // 4, 4 * bx + s % 4, c])
                    if a == b:
                        code = 0
                    else:
                        jj = j if a > b else 7 - j
                        code = 0 if jj == 0 else (1 if jj == 7 else jj + 1)
                    field |= code << (3 * s)
                e0, e1 = (a, b) if a >= b else (b, a)
                out[by, bx, c, 0] = e0
                out[by, bx, c, 1] = e1
                for k in range(6):
                    out[by, bx, c, 2 + k] = (field >> (8 * k)) & 0xFF
    return out


# --------------------------------------------------------------------------------------
# Training of the hybrid layout (Sec. 3.4, Eq. 6-7 and its noise equation; Sec. 4)
# --------------------------------------------------------------------------------------
# State (float32 master copies, one array per key):
#   fuv_ep [H/4][W/4][4][2], fuv_w [H][W][4]            F_uv as block endpoints and weights
#   fuvt_ep [S][Gv/4][Gu/4][4][2], fuvt_w [S][Gv][Gu][4]  F_uvt slices, the same way
#   fut [Tt][U][2], fvt [Tt][V][2]                       8-bit planes (trained in float)
#   mlp [hybrid_mlp_size(hidden)]
# (fuv_w [H][W] and fuvt_w [S][Gv][Gu] with codec 1: one weight per texel, Eq. (6)).
# A training sample is texel (x, y) of baked frame i (time keys[i], or i / (n - 1) with no
# key table), so tau = i / (n - 1).  Flags (readings):
# * none: F_uv / F_uvt are the continuous Eq. (7) lerp of their endpoints and weights.
#   This is the paper's BC simulation: the maps are parameterised by a block's two
#   endpoints and per-texel weights during training (Sec. 3.4; supplementary ablation,
#   "w/ BC simulation").
# * NOISE adds U(-1/2, 1/2) / 256 to each of the 12 sampled map values (Sec. 3.4's noise
#   equation for V_ut and V_vt, alpha = 1/256; the same text adds noise to the sampled V_uvt
#   and V_uv).
# * DIRECT: F_uv / F_uvt are per-texel values, the state's weights themselves (codec 0
#   layout, one value per texel and channel; endpoints unused).  This is the supplementary
#   ablation's "w/o BC simulation" arm, a directly optimised feature map that is
#   block-compressed only after training (hybrid_encode).
# * BCSIM rounds the endpoints and weights to the block format's grid during training (8-bit
#   endpoints and 3-bit weights for BC4, R12; mode-6 endpoints and 4-bit weights for BC7)
#   with the straight-through gradient (R14).  The paper does not describe rounding during
#   training; it is kept as a variant, and for fine-tuning the decoder on features that are
#   exactly the exported blocks' decode.
# * QPLANES feeds F_ut / F_vt rounded to 8 bits, the values a decode sees (used to fine-tune
#   the decoder on frozen features, Sec. 4).
# * the noise of sample s, channel c in step `step` is a counter-based draw: the 64-bit
#   SplitMix64 output function (Steele, Lea, Flood 2014) applied to
#   seed * 0x9E3779B97F4A7C15 + step * 2^32 + s * 16 + c; its top 24 bits / 2^24 - 1/2.
HT_BCSIM, HT_NOISE, HT_QPLANES, HT_DIRECT = 1, 2, 4, 8
NOISE_ALPHA = 1.0 / 256.0
_M64 = (1 << 64) - 1


def splitmix64(x):
    """SplitMix64 output function on uint64 (numpy arrays wrap modulo 2^64)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = x + np.uint64(0x9E3779B97F4A7C15)
        x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return x ^ (x >> np.uint64(31))


def hybrid_noise(seed: int, step: int, s, c) -> np.ndarray:
    """U(-1/2, 1/2) draws of samples s, channels c (broadcast) in one step."""
    base = np.uint64((seed * 0x9E3779B97F4A7C15 + (step << 32)) & _M64)
    with np.errstate(over="ignore"):
        ctr = base + (np.asarray(s, dtype=np.uint64) * np.uint64(16) + np.asarray(c, dtype=np.uint64))
    top = (splitmix64(ctr) >> np.uint64(40)).astype(np.float64)
    return top / float(1 << 24) - 0.5


def _bc_texels(ep, wt, sl, ys, xs, bcsim: bool, codec: int = 0, direct: bool = False):
    """4-channel texels of a block-parameterised map at (ys, xs) (and slice sl, or None):
    (value in [0, 1], d/de1, d/de2, d/dw) per channel.  codec 0: one weight per channel
    (BC4 per channel); codec 1: one weight per texel shared by the 4 channels (BC7 mode 6,
    Eq. (6)), whose gradient is the sum over channels of dw.  direct: the weights are the
    texel values themselves (codec 0 layout)."""
    if sl is None:
        e = ep[ys >> 2, xs >> 2]            # [..., 4, 2]
        w = wt[ys, xs]                      # [..., 4] or [...]
    else:
        e = ep[sl, ys >> 2, xs >> 2]
        w = wt[sl, ys, xs]
    if direct:
        assert codec == 0, "a directly optimised map keeps one value per texel and channel"
        zero = np.zeros(np.shape(w))
        return np.asarray(w, dtype=np.float64), zero, zero, np.ones(np.shape(w))
    if codec == 1:
        w = np.repeat(np.asarray(w)[..., None], 4, axis=-1)
        if bcsim:
            E1 = bc7_quantise_endpoint(e[..., 0])[0].astype(np.float64)
            E2 = bc7_quantise_endpoint(e[..., 1])[0].astype(np.float64)
            J = quantise_weight4(w)
            wj = np.asarray(BC7_WEIGHTS4, dtype=np.int64)[J].astype(np.float64)
            val = np.floor(((64 - wj) * E1 + wj * E2 + 32) / 64) / 255.0
            return val, 1.0 - wj / 64.0, wj / 64.0, (E2 - E1) / 255.0
    if bcsim:
        E1 = quantise_endpoint(e[..., 0]).astype(np.float64)
        E2 = quantise_endpoint(e[..., 1]).astype(np.float64)
        J = quantise_weight(w).astype(np.float64)
        val = bcsim_value(E1.astype(np.int64), E2.astype(np.int64), J.astype(np.int64)) / 255.0
        return val, 1.0 - J / 7.0, J / 7.0, (E2 - E1) / 255.0
    e1 = e[..., 0].astype(np.float64)
    e2 = e[..., 1].astype(np.float64)
    w = w.astype(np.float64)
    return (1.0 - w) * e1 + w * e2, 1.0 - w, w, e2 - e1


def hybrid_train_forward(state: dict, xs, ys, fs, flags: int, seed: int = 0, step: int = 0,
                         need_cache: bool = False, s_offset: int = 0):
    """Decoder output at training samples (texel (x, y) of frame f) -> [B][3].  The noise
    counter of sample j is s_offset + j (its position in the whole batch)."""
    d = state["dims"]
    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    fs = np.asarray(fs, dtype=np.int64)
    nf = d["frames"]
    tau = fs / (nf - 1) if nf > 1 else np.zeros(fs.shape)
    keys = np.asarray(d["keys"], dtype=np.float64)
    t = keys[fs] if keys.size else tau
    bc = bool(flags & HT_BCSIM)
    direct = bool(flags & HT_DIRECT)
    assert not (bc and direct), "BCSIM and DIRECT exclude each other"
    codec = d.get("codec", 0)
    u = (xs + 0.5) / d["W"]
    v = (ys + 0.5) / d["H"]
    taps = {}
    # V_uvt
    gx0, gx1, wx0, wx1 = _axis(u, d["Gu"])
    gy0, gy1, wy0, wy1 = _axis(v, d["Gv"])
    s0, s1, ws0, ws1 = _node_axis(tau, d["S"])
    Vuvt = np.zeros(xs.shape + (4,))
    taps["uvt"] = []
    for (ss, ws) in ((s0, ws0), (s1, ws1)):
        for (yy, wy) in ((gy0, wy0), (gy1, wy1)):
            for (xx, wx) in ((gx0, wx0), (gx1, wx1)):
                val, d1, d2, dw = _bc_texels(state["fuvt_ep"], state["fuvt_w"], ss, yy, xx, bc, codec, direct)
                w = ws * wy * wx
                Vuvt += w[..., None] * val
                taps["uvt"].append((ss, yy, xx, w, d1, d2, dw))
    # V_uv: the texel itself
    val, d1, d2, dw = _bc_texels(state["fuv_ep"], state["fuv_w"], None, ys, xs, bc, codec, direct)
    Vuv = val
    taps["uv"] = (d1, d2, dw)
    # planes
    k0, k1, wk0, wk1 = _node_axis(tau, d["Tt"])
    planes = []
    taps["planes"] = []
    for (c, size, key) in ((u, d["U"], "fut"), (v, d["V"], "fvt")):
        a0, a1, wa0, wa1 = _axis(c, size)
        P = np.zeros(xs.shape + (2,))
        arr = np.asarray(state[key], dtype=np.float64)
        if flags & HT_QPLANES:
            arr = np.rint(np.float32(255.0) * np.asarray(state[key], dtype=np.float32)).astype(np.float64) / 255.0
        lst = []
        for (kk, wk) in ((k0, wk0), (k1, wk1)):
            for (aa, wa) in ((a0, wa0), (a1, wa1)):
                P += (wk * wa)[..., None] * arr[kk, aa]
                lst.append((kk, aa, wk * wa))
        planes.append(P)
        taps["planes"].append(lst)
    x = np.concatenate([Vuvt, Vuv, planes[0], planes[1], gamma_t(t)], axis=-1)
    if flags & HT_NOISE:
        sidx = s_offset + np.arange(xs.size).reshape(xs.shape)
        x[..., :12] += NOISE_ALPHA * hybrid_noise(seed, step, sidx[..., None], np.arange(12))
    P = unpack_hybrid_mlp(state["mlp"], d["hidden"])
    a1 = x @ P["W1"].T + P["b1"]
    h1 = gelu(a1)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = gelu(a2)
    out = h2 @ P["W3"].T + P["b3"]
    if not need_cache:
        return out
    return out, dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2, P=P, taps=taps)


def gelu_grad(a: np.ndarray) -> np.ndarray:
    """d GELU / da = Phi(a) + a phi(a)."""
    from scipy.special import erf
    a = np.asarray(a, dtype=np.float64)
    return 0.5 * (1.0 + erf(a / np.sqrt(2.0))) + a * np.exp(-0.5 * a * a) / np.sqrt(2.0 * np.pi)


def hybrid_train_grads(state: dict, xs, ys, fs, target, flags: int, seed: int = 0, step: int = 0,
                       s_offset: int = 0):
    """L2 loss (mean over this model's samples and channels) and its gradients for every
    state array.  Reading (several per-tile models trained together): each model's loss is
    the mean over its own samples, so a model's gradients do not depend on how many other
    models share the launch (Adam is not invariant to a common gradient scale, through its
    epsilon); the loss reported for the launch is the mean of the models' losses.  This
    model's samples start at position s_offset of the batch (their noise counters)."""
    d = state["dims"]
    codec = d.get("codec", 0)
    out, c = hybrid_train_forward(state, xs, ys, fs, flags, seed, step, need_cache=True, s_offset=s_offset)
    target = np.asarray(target, dtype=np.float64)
    n = out.size
    loss = float(np.sum((out - target) ** 2) / n)
    P = c["P"]
    dout = (2.0 / n) * (out - target)
    gW3, gb3 = dout.T @ c["h2"], dout.sum(0)
    da2 = (dout @ P["W3"]) * gelu_grad(c["a2"])
    gW2, gb2 = da2.T @ c["h1"], da2.sum(0)
    da1 = (da2 @ P["W2"]) * gelu_grad(c["a1"])
    gW1, gb1 = da1.T @ c["x"], da1.sum(0)
    dx = da1 @ P["W1"]
    g = {k: np.zeros(np.asarray(state[k]).shape) for k in ("fuv_ep", "fuv_w", "fuvt_ep", "fuvt_w", "fut", "fvt")}
    g["mlp"] = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    xs = np.asarray(xs, dtype=np.int64)
    ys = np.asarray(ys, dtype=np.int64)
    ch = np.arange(4)[None, :]
    for (ss, yy, xx, w, d1, d2, dw) in c["taps"]["uvt"]:
        dv = w[:, None] * dx[:, 0:4]
        sl, by, bx = ss[:, None], (yy >> 2)[:, None], (xx >> 2)[:, None]
        np.add.at(g["fuvt_ep"], (sl, by, bx, ch, 0), dv * d1)
        np.add.at(g["fuvt_ep"], (sl, by, bx, ch, 1), dv * d2)
        if codec == 1:
            np.add.at(g["fuvt_w"], (ss, yy, xx), (dv * dw).sum(-1))
        else:
            np.add.at(g["fuvt_w"], (sl, yy[:, None], xx[:, None], ch), dv * dw)
    d1, d2, dw = c["taps"]["uv"]
    dv = dx[:, 4:8]
    np.add.at(g["fuv_ep"], ((ys >> 2)[:, None], (xs >> 2)[:, None], ch, 0), dv * d1)
    np.add.at(g["fuv_ep"], ((ys >> 2)[:, None], (xs >> 2)[:, None], ch, 1), dv * d2)
    if codec == 1:
        np.add.at(g["fuv_w"], (ys, xs), (dv * dw).sum(-1))
    else:
        np.add.at(g["fuv_w"], (ys[:, None], xs[:, None], ch), dv * dw)
    for pi, key in enumerate(("fut", "fvt")):
        dv = dx[:, 8 + 2 * pi: 10 + 2 * pi]
        for (kk, aa, w) in c["taps"]["planes"][pi]:
            np.add.at(g[key], (kk[:, None], aa[:, None], np.arange(2)[None, :]), w[:, None] * dv)
    return loss, g


HYB_KEYS = ("fuv_ep", "fuv_w", "fuvt_ep", "fuvt_w", "fut", "fvt", "mlp")


def hybrid_train_step(state: dict, opt: dict, xs, ys, fs, target, flags: int, seed: int = 0):
    """Forward, L2 loss, backward, Adam on every array (lr_feat for the feature maps,
    lr_mlp for the decoder), feature maps projected to [0, 1].  Returns the loss."""
    loss, g = hybrid_train_grads(state, xs, ys, fs, target, flags, seed, opt["step"])
    opt["step"] += 1
    for key in HYB_KEYS:
        lr = opt["lr_mlp"] if key == "mlp" else opt["lr_feat"]
        p, m, v = adam_update(state[key], g[key], opt["m"][key], opt["v"][key], opt["step"], lr)
        if key != "mlp":
            p = np.clip(p, 0.0, 1.0)
        state[key], opt["m"][key], opt["v"][key] = p, m, v
    return loss


def hybrid_normalise_target(target: np.ndarray, gamma: float):
    """Sec. 4 preprocessing: gamma correction y^(1/gamma), then per frame and channel
    division by the mean.  target [n][H][W][3] (FP16 values read exactly) -> (normalised
    [n][H][W][3], means [n][3])."""
    y = np.asarray(target, dtype=np.float64) ** (1.0 / gamma)
    means = y.mean(axis=(1, 2))
    return y / means[:, None, None, :], means


def hybrid_restore(pred: np.ndarray, mean3, gamma: float) -> np.ndarray:
    """Inverse of the preprocessing for one frame: (pred * mean)^gamma (negative products
    clamp to 0)."""
    return np.maximum(np.asarray(pred, dtype=np.float64) * np.asarray(mean3, dtype=np.float64), 0.0) ** gamma


def hybrid_export(state: dict) -> dict:
    """Decodable hybrid model of a trained state: BC4 blocks of F_uv and of each F_uvt
    slice (export_bc4), planes rounded to 8 bits (rint of the float32 product 255 v)."""
    d = state["dims"]
    codec = d.get("codec", 0)
    enc = export_bc7 if codec == 1 else export_bc4
    fuvt = np.stack([enc(state["fuvt_ep"][s], state["fuvt_w"][s]) for s in range(d["S"])])
    q = lambda a: np.rint(np.float32(255.0) * np.asarray(a, dtype=np.float32)).astype(np.uint8)
    return dict(W=d["W"], H=d["H"], Gu=d["Gu"], Gv=d["Gv"], S=d["S"], U=d["U"], V=d["V"], Tt=d["Tt"],
                hidden=d["hidden"], codec=codec, fuv=enc(state["fuv_ep"], state["fuv_w"]), fuvt=fuvt,
                fut=q(state["fut"]), fvt=q(state["fvt"]), keys=np.asarray(d["keys"], dtype=np.float32),
                mlp=np.asarray(state["mlp"], dtype=np.float32))


# --------------------------------------------------------------------------------------
# Block encoders from texel values, and the paper's export path (Sec. 3.4)
# --------------------------------------------------------------------------------------
# After training the paper reconstructs F_uv and F_uvt from the learned parameters,
# quantises them to 8 bits and block-compresses the result (Sec. 3.4, last paragraph of
# "Feature Map Compression"); the "w/o BC simulation" ablation arm compresses a directly
# optimised map the same way (supplementary ablation study).  The paper names no encoder.
# Readings:
# * BC4: the block nearest to the 16 texels in summed squared error, found by trying every
#   one of the 65536 endpoint pairs (both palette modes of R1) with each texel's best
#   selector; ties go to the lowest e0 * 256 + e1, and per texel to the lowest selector.
#   Exhaustive, so it is the optimum.
# * BC7 mode 6: 2^58 endpoint settings are too many to try, so the encoder is a fixed,
#   integer-only search (identical steps run on the GPU):
#     1. endpoints at the corners of the texels' bounding box along its principal
#        diagonal: the channel of largest spread is the reference, and each other channel
#        runs from its minimum to its maximum when its covariance with the reference is
#        >= 0, else from maximum to minimum;
#     2. every target endpoint is quantised for each of the four p-bit pairs
#        (v = clamp(floor((x - p + 1) / 2), 0, 127), endpoint 2 v + p); each texel takes its
#        best 4-bit index (lowest index on ties) and the pair of least summed squared error
#        is kept (a candidate replaces the current one only if strictly better);
#     3. twice: the least-squares endpoints for the current indices (per channel, the 2x2
#        normal equations of sum ((64 - w) E0 + w E1 - 64 x)^2, solved exactly and rounded
#        half up, clamped to 0..255), quantised as in 2;
#     4. best-improvement local search at step sizes s = 8, 4, 2, 1 in turn: 22 moves (each
#        7-bit value of each endpoint -s and +s; all 4 values of one endpoint -s and +s
#        together; each p-bit flipped; a move leaving 0..127 is not taken), indices refitted
#        per move; the best move is taken while it is strictly better (ties between moves
#        go to the first in that order), at most 64 rounds per step size;
#     5. when texel 0's index has its top bit set, the endpoints swap and each index J
#        becomes 15 - J (the anchor index has 3 bits; the decode is unchanged).
#   Exact on blocks that one mode-6 block reproduces when the block uses indices 0 and 15;
#   pinned by brute force on small cases (tests).

def encode_bc4(texels) -> np.ndarray:
    """BC4 blocks [n][8] of 8-bit texels [n][16] (texel s = 4 row + col): the exhaustive
    search described above."""
    X = np.asarray(texels, dtype=np.int64).reshape(-1, 16)
    pair = np.arange(65536, dtype=np.int64)
    code = np.arange(8, dtype=np.int64)
    pal = bc4_palette_value((pair >> 8)[:, None], (pair & 255)[:, None], code[None, :]).astype(np.int64)
    out = np.zeros((X.shape[0], 8), dtype=np.uint8)
    for b in range(X.shape[0]):
        vals, counts = np.unique(X[b], return_counts=True)
        d = (pal[:, None, :] - vals[None, :, None]) ** 2          # [pairs][distinct values][codes]
        sse = (d.min(-1) * counts[None, :]).sum(-1)
        p = int(np.argmin(sse))                                    # first minimum: lowest pair
        e0, e1 = p >> 8, p & 255
        dp = (pal[p][None, :] - X[b][:, None]) ** 2                # [16][codes]
        codes = dp.argmin(-1)                                      # lowest code on ties
        field = 0
        for s_ in range(16):
            field |= int(codes[s_]) << (3 * s_)
        out[b, 0], out[b, 1] = e0, e1
        for k in range(6):
            out[b, 2 + k] = (field >> (8 * k)) & 0xFF
    return out


_W4 = np.asarray(BC7_WEIGHTS4, dtype=np.int64)
BC7_SEARCH_STEPS = (8, 4, 2, 1)
BC7_SEARCH_ROUNDS = 64


def _m6_fit(X, E0, E1):
    """Best 4-bit index of every texel for endpoints E0, E1 [nb][4]: (J [nb][16], sse [nb])."""
    pal = ((64 - _W4)[None, :, None] * E0[:, None, :] + _W4[None, :, None] * E1[:, None, :] + 32) >> 6
    d = ((pal[:, None, :, :] - X[:, :, None, :]) ** 2).sum(-1)     # [nb][texel][index]
    return d.argmin(-1), d.min(-1).sum(-1)


def _m6_q7(x, p):
    """7-bit value of target x [nb][4] for p-bit p [nb]."""
    return np.clip((x - p[:, None] + 1) >> 1, 0, 127)


def encode_bc7m6(texels) -> np.ndarray:
    """BC7 mode-6 blocks [n][16] of 8-bit RGBA texels [n][16][4]: the search described above."""
    X = np.asarray(texels, dtype=np.int64).reshape(-1, 16, 4)
    nb = X.shape[0]
    rows = np.arange(nb)
    big = np.iinfo(np.int64).max
    cur = dict(v0=np.zeros((nb, 4), np.int64), p0=np.zeros(nb, np.int64), v1=np.zeros((nb, 4), np.int64),
               p1=np.zeros(nb, np.int64), J=np.zeros((nb, 16), np.int64), sse=np.full(nb, big))

    def take(v0, p0, v1, p1):
        J, sse = _m6_fit(X, 2 * v0 + p0[:, None], 2 * v1 + p1[:, None])
        t = sse < cur["sse"]
        for k, val in (("v0", v0), ("p0", p0), ("v1", v1), ("p1", p1), ("J", J), ("sse", sse)):
            cur[k] = np.where(t[:, None], val, cur[k]) if val.ndim == 2 else np.where(t, val, cur[k])

    def quantised(A, B):
        for q0, q1 in ((0, 0), (0, 1), (1, 0), (1, 1)):
            p0, p1 = np.full(nb, q0, np.int64), np.full(nb, q1, np.int64)
            take(_m6_q7(A, p0), p0, _m6_q7(B, p1), p1)

    # 1-2: bounding-box diagonal
    D = 16 * X - X.sum(1, keepdims=True)
    var = (D * D).sum(1)
    ref = var.argmax(-1)
    cov = (D * D[rows, :, ref][:, :, None]).sum(1)
    lo, hi = X.min(1), X.max(1)
    pos = cov >= 0
    quantised(np.where(pos, lo, hi), np.where(pos, hi, lo))
    # 3: least-squares endpoints for the current indices, twice
    for _ in range(2):
        w = _W4[cur["J"]]
        a, b = 64 - w, w
        Aa, Bab, Cb = (a * a).sum(1), (a * b).sum(1), (b * b).sum(1)
        r0 = 64 * (a[:, :, None] * X).sum(1)
        r1 = 64 * (b[:, :, None] * X).sum(1)
        det = Aa * Cb - Bab * Bab
        ok = det > 0
        dd = np.where(ok, det, 1)[:, None]
        n0 = Cb[:, None] * r0 - Bab[:, None] * r1
        n1 = Aa[:, None] * r1 - Bab[:, None] * r0
        E0 = np.clip(np.floor_divide(2 * n0 + dd, 2 * dd), 0, 255)
        E1 = np.clip(np.floor_divide(2 * n1 + dd, 2 * dd), 0, 255)
        E0 = np.where(ok[:, None], E0, 2 * cur["v0"] + cur["p0"][:, None])
        E1 = np.where(ok[:, None], E1, 2 * cur["v1"] + cur["p1"][:, None])
        quantised(E0, E1)
    # 4: local search, coarse to fine
    for st in BC7_SEARCH_STEPS:
        moves = ([(k, c, dv) for k in (0, 1) for c in range(4) for dv in (-st, st)] +
                 [(k, 4, dv) for k in (0, 1) for dv in (-st, st)] + [(0, -1, 0), (1, -1, 0)])
        for _ in range(BC7_SEARCH_ROUNDS):
            cand = []
            for (k, c, dv) in moves:
                v0, p0, v1, p1 = cur["v0"].copy(), cur["p0"].copy(), cur["v1"].copy(), cur["p1"].copy()
                if c >= 0:
                    v = v0 if k == 0 else v1
                    cols = slice(None) if c == 4 else slice(c, c + 1)
                    v[:, cols] += dv
                    valid = ((v[:, cols] >= 0) & (v[:, cols] <= 127)).all(1)
                    np.clip(v, 0, 127, out=v)
                else:
                    valid = np.ones(nb, bool)
                    if k == 0:
                        p0 = 1 - p0
                    else:
                        p1 = 1 - p1
                J, sse = _m6_fit(X, 2 * v0 + p0[:, None], 2 * v1 + p1[:, None])
                cand.append((np.where(valid, sse, big), v0, p0, v1, p1, J))
            S = np.stack([c_[0] for c_ in cand], axis=1)
            best = S.argmin(1)
            better = S[rows, best] < cur["sse"]
            if not better.any():
                break
            for i, (sse, v0, p0, v1, p1, J) in enumerate(cand):
                t = better & (best == i)
                for kk, val in (("v0", v0), ("p0", p0), ("v1", v1), ("p1", p1), ("J", J), ("sse", sse)):
                    cur[kk] = np.where(t[:, None], val, cur[kk]) if val.ndim == 2 else np.where(t, val, cur[kk])
    # 5: anchor and packing
    out = np.zeros((nb, 16), dtype=np.uint8)
    for i in range(nb):
        a, b, pa, pb = cur["v0"][i], cur["v1"][i], int(cur["p0"][i]), int(cur["p1"][i])
        idx = [int(j) for j in cur["J"][i]]
        if idx[0] >= 8:
            a, b, pa, pb = b, a, pb, pa
            idx = [15 - j for j in idx]
        bits = 0x40
        for c in range(4):
            bits |= int(a[c]) << (7 + 14 * c)
            bits |= int(b[c]) << (14 + 14 * c)
        bits |= pa << 63
        bits |= pb << 64
        bits |= idx[0] << 65
        for s_ in range(1, 16):
            bits |= idx[s_] << (64 + 4 * s_)
        out[i] = np.frombuffer(bits.to_bytes(16, "little"), dtype=np.uint8)
    return out


# BC7 with several modes (Sec. 3.4: the BC7 compression may pick among the format's modes): every
# block tries mode 6 (the search above), mode 5 under each of its 4 rotations and mode 4
# under each rotation and both index selections, and keeps the candidate of least summed
# squared error over its 16 texels and 4 channels (ties: mode 6, then mode 5 by rotation,
# then mode 4 by rotation then selection).  A rotation r > 0 encodes the texels with channel
# r - 1 and channel 3 exchanged (the decoder exchanges them back).  Modes 5 and 4 fit their
# colour (3 channels) and alpha (1 channel) endpoints apart, each with the same fixed search
# at its own endpoint precision n and index width b (mode 5: 7 / 2 and 8 / 2; mode 4: 5 / b
# and 6 / b' with (b, b') = (2, 3), or (3, 2) under selection 1):
#   1. endpoints at the bounding-box diagonal as in step 1 above (one channel: its minimum
#      and maximum), each 8-bit target x quantised to the n-bit value whose expansion is
#      nearest (ties to the lower value; the candidates are round(x (2^n - 1) / 255) and
#      its two neighbours);
#   2. twice: least-squares endpoints for the current indices as in step 3 above, quantised
#      as in 1;
#   3. best-improvement local search at step sizes 2^(n - 4), ..., 2, 1: each value of each
#      endpoint -s and +s, then (several channels only) all values of one endpoint -s and
#      +s, a move leaving 0 .. 2^n - 1 not taken, at most 64 rounds per step size;
#   4. when texel 0's index has its top bit set, the endpoints swap and each index J becomes
#      2^b - 1 - J (the weight tables are symmetric).
# Every candidate's indices are refitted (each texel its least-error index, the lowest on
# ties) and a candidate replaces the current one only when strictly better.
def _bc7_q(x, n: int):
    """n-bit values whose expansion is nearest to the 8-bit targets x (ties to the lower)."""
    x = np.asarray(x, dtype=np.int64)
    top = (1 << n) - 1
    g = np.clip((x * top + 127) // 255, 0, top)
    best, bd = None, None
    for dv in (-1, 0, 1):
        v = np.clip(g + dv, 0, top)
        d = np.abs(((v << (8 - n)) | (v >> (2 * n - 8)) if n < 8 else v) - x)
        if best is None:
            best, bd = v, d
        else:
            t = (d < bd) | ((d == bd) & (v < best))
            best, bd = np.where(t, v, best), np.where(t, d, bd)
    return best


def _bc7_x(v, n: int):
    return ((v << (8 - n)) | (v >> (2 * n - 8))) if n < 8 else v


def _sub_search(X, n: int, ib: int):
    """The fixed search for one endpoint pair of n-bit values and b-bit indices over texels
    X [nb][16][C] (8-bit): (v0 [nb][C], v1 [nb][C], J [nb][16], sse [nb])."""
    nb, _, C = X.shape
    rows = np.arange(nb)
    Wt = np.asarray(BC7_WEIGHTS[ib], dtype=np.int64)
    top = (1 << n) - 1
    big = np.iinfo(np.int64).max
    cur = dict(v0=np.zeros((nb, C), np.int64), v1=np.zeros((nb, C), np.int64), J=np.zeros((nb, 16), np.int64),
               sse=np.full(nb, big))

    def fit(v0, v1):
        E0, E1 = _bc7_x(v0, n), _bc7_x(v1, n)
        pal = ((64 - Wt)[None, :, None] * E0[:, None, :] + Wt[None, :, None] * E1[:, None, :] + 32) >> 6
        d = ((pal[:, None, :, :] - X[:, :, None, :]) ** 2).sum(-1)
        return d.argmin(-1), d.min(-1).sum(-1)

    def take(v0, v1):
        J, sse = fit(v0, v1)
        t = sse < cur["sse"]
        for k, val in (("v0", v0), ("v1", v1), ("J", J), ("sse", sse)):
            cur[k] = np.where(t[:, None], val, cur[k]) if val.ndim == 2 else np.where(t, val, cur[k])
    # 1
    lo, hi = X.min(1), X.max(1)
    if C > 1:
        D = 16 * X - X.sum(1, keepdims=True)
        ref = (D * D).sum(1).argmax(-1)
        pos = (D * D[rows, :, ref][:, :, None]).sum(1) >= 0
    else:
        pos = np.ones((nb, 1), bool)
    take(_bc7_q(np.where(pos, lo, hi), n), _bc7_q(np.where(pos, hi, lo), n))
    # 2
    for _ in range(2):
        w = Wt[cur["J"]]
        a, b = 64 - w, w
        Aa, Bab, Cb = (a * a).sum(1), (a * b).sum(1), (b * b).sum(1)
        r0, r1 = 64 * (a[:, :, None] * X).sum(1), 64 * (b[:, :, None] * X).sum(1)
        det = Aa * Cb - Bab * Bab
        ok = det > 0
        dd = np.where(ok, det, 1)[:, None]
        E0 = np.clip(np.floor_divide(2 * (Cb[:, None] * r0 - Bab[:, None] * r1) + dd, 2 * dd), 0, 255)
        E1 = np.clip(np.floor_divide(2 * (Aa[:, None] * r1 - Bab[:, None] * r0) + dd, 2 * dd), 0, 255)
        E0 = np.where(ok[:, None], E0, _bc7_x(cur["v0"], n))
        E1 = np.where(ok[:, None], E1, _bc7_x(cur["v1"], n))
        take(_bc7_q(E0, n), _bc7_q(E1, n))
    # 3
    for st in [1 << e for e in range(n - 4, -1, -1)]:
        moves = [(k, c, dv) for k in (0, 1) for c in range(C) for dv in (-st, st)]
        if C > 1:
            moves += [(k, C, dv) for k in (0, 1) for dv in (-st, st)]
        for _ in range(BC7_SEARCH_ROUNDS):
            cand = []
            for (k, c, dv) in moves:
                v0, v1 = cur["v0"].copy(), cur["v1"].copy()
                v = v0 if k == 0 else v1
                cols = slice(None) if c == C else slice(c, c + 1)
                v[:, cols] += dv
                valid = ((v[:, cols] >= 0) & (v[:, cols] <= top)).all(1)
                np.clip(v, 0, top, out=v)
                J, sse = fit(v0, v1)
                cand.append((np.where(valid, sse, big), v0, v1, J))
            S = np.stack([c_[0] for c_ in cand], axis=1)
            best = S.argmin(1)
            better = S[rows, best] < cur["sse"]
            if not better.any():
                break
            for i, (sse, v0, v1, J) in enumerate(cand):
                t = better & (best == i)
                for kk, val in (("v0", v0), ("v1", v1), ("J", J), ("sse", sse)):
                    cur[kk] = np.where(t[:, None], val, cur[kk]) if val.ndim == 2 else np.where(t, val, cur[kk])
    # 4
    sw = cur["J"][:, 0] >= (1 << (ib - 1))
    v0 = np.where(sw[:, None], cur["v1"], cur["v0"])
    v1 = np.where(sw[:, None], cur["v0"], cur["v1"])
    J = np.where(sw[:, None], (1 << ib) - 1 - cur["J"], cur["J"])
    return v0, v1, J, cur["sse"]


def _pack_set(bits: int, pos: int, J, b: int) -> tuple:
    bits |= int(J[0]) << pos
    pos += b - 1
    for s_ in range(1, 16):
        bits |= int(J[s_]) << pos
        pos += b
    return bits, pos


def _bc7_rotated(X, r: int):
    if r == 0:
        return X
    Y = X.copy()
    Y[..., r - 1], Y[..., 3] = X[..., 3], X[..., r - 1]
    return Y


def encode_bc7(texels) -> np.ndarray:
    """BC7 blocks [n][16] of 8-bit 4-channel texels [n][16][4] using modes 6, 5 and 4: the
    per-block choice described above."""
    X = np.asarray(texels, dtype=np.int64).reshape(-1, 16, 4)
    nb = X.shape[0]
    m6 = encode_bc7m6(X)
    sse6 = ((np.stack([bc7m6_decode_block(b) for b in m6]).astype(np.int64) - X) ** 2).sum((1, 2))
    best = [("m6", i) for i in range(nb)]
    best_sse = sse6.copy()
    cands = []
    for r in range(4):
        Y = _bc7_rotated(X, r)
        cands.append((5, r, 0, _sub_search(Y[..., :3], 7, 2), _sub_search(Y[..., 3:], 8, 2)))
    for r in range(4):
        Y = _bc7_rotated(X, r)
        for sel in (0, 1):
            cb, ab = (2, 3) if sel == 0 else (3, 2)
            cands.append((4, r, sel, _sub_search(Y[..., :3], 5, cb), _sub_search(Y[..., 3:], 6, ab)))
    choice = np.full(nb, -1)
    for ci, (_, _, _, col, alp) in enumerate(cands):
        sse = col[3] + alp[3]
        t = sse < best_sse
        best_sse = np.where(t, sse, best_sse)
        choice = np.where(t, ci, choice)
    out = m6.copy()
    for i in range(nb):
        if choice[i] < 0:
            continue
        mode, r, sel, col, alp = cands[choice[i]]
        cv0, cv1, cJ = col[0][i], col[1][i], col[2][i]
        av0, av1, aJ = alp[0][i], alp[1][i], alp[2][i]
        if mode == 5:
            bits = (1 << 5) | (r << 6)
            for c in range(3):
                bits |= int(cv0[c]) << (8 + 14 * c)
                bits |= int(cv1[c]) << (15 + 14 * c)
            bits |= int(av0[0]) << 50
            bits |= int(av1[0]) << 58
            bits, _ = _pack_set(bits, 66, cJ, 2)
            bits, _ = _pack_set(bits, 97, aJ, 2)
        else:
            bits = (1 << 4) | (r << 5) | (sel << 7)
            for c in range(3):
                bits |= int(cv0[c]) << (8 + 10 * c)
                bits |= int(cv1[c]) << (13 + 10 * c)
            bits |= int(av0[0]) << 38
            bits |= int(av1[0]) << 44
            s2, s3 = (cJ, aJ) if sel == 0 else (aJ, cJ)
            bits, _ = _pack_set(bits, 50, s2, 2)
            bits, _ = _pack_set(bits, 81, s3, 3)
        out[i] = np.frombuffer(bits.to_bytes(16, "little"), dtype=np.uint8)
    return out


def _map_texels_u8(ep, wt, flags: int, codec: int) -> np.ndarray:
    """8-bit texels [..][H][W][4] of a block-parameterised map (endpoints [..][H/4][W/4][4][2],
    weights [..][H][W][4] or, codec 1, [..][H][W]) as training with `flags` reads it: the
    simulated texel under BCSIM; else the value v (the weight itself under DIRECT, the float32
    Eq. (7) lerp fl32(fl32(fl32(1 - w) e1) + fl32(w e2)) otherwise) quantised as
    clamp(rint(fl32(255 v)), 0, 255)."""
    ep = np.asarray(ep, dtype=np.float32)
    wt = np.asarray(wt, dtype=np.float32)
    if codec == 1:
        wt = np.repeat(wt[..., None], 4, axis=-1)
    e = np.repeat(np.repeat(ep, 4, axis=-4), 4, axis=-3)          # [..][H][W][4][2]
    if flags & HT_BCSIM:
        if codec == 1:
            E1 = bc7_quantise_endpoint(ep[..., 0])[0]
            E2 = bc7_quantise_endpoint(ep[..., 1])[0]
            E1 = np.repeat(np.repeat(E1, 4, axis=-3), 4, axis=-2)
            E2 = np.repeat(np.repeat(E2, 4, axis=-3), 4, axis=-2)
            w = _W4[quantise_weight4(wt)]
            return ((64 - w) * E1 + w * E2 + 32) >> 6
        return bcsim_value(quantise_endpoint(e[..., 0]), quantise_endpoint(e[..., 1]), quantise_weight(wt))
    if flags & HT_DIRECT:
        v = wt
    else:
        one = np.float32(1.0)
        v = ((one - wt) * e[..., 0]) + (wt * e[..., 1])            # float32 throughout
    return np.clip(np.rint(np.float32(255.0) * v), 0, 255).astype(np.int64)


def _footprints(tex):
    """[..][H][W][4] texels -> [..][H/4][W/4][16][4] (texel s = 4 row + col)."""
    sh = tex.shape
    t = tex.reshape(sh[:-3] + (sh[-3] // 4, 4, sh[-2] // 4, 4, 4))
    n = len(sh) - 3
    t = np.moveaxis(t, n + 2, n + 1)                               # [..][Hb][Wb][4 rows][4 cols][4]
    return t.reshape(sh[:-3] + (sh[-3] // 4, sh[-2] // 4, 16, 4))


def encode_map(tex, codec: int) -> np.ndarray:
    """Blocks of an 8-bit 4-channel map [..][H][W][4]: BC7 of modes 6, 5 and 4 (encode_bc7;
    [..][H/4][W/4][16], codec 1) or one BC4 block per channel ([..][H/4][W/4][4][8], codec 0)."""
    fp = _footprints(np.asarray(tex, dtype=np.int64))
    lead = fp.shape[:-2]
    if codec == 1:
        return encode_bc7(fp.reshape(-1, 16, 4)).reshape(lead + (16,))
    per_ch = np.moveaxis(fp, -1, -2)                               # [..][Hb][Wb][4 ch][16]
    return encode_bc4(per_ch.reshape(-1, 16)).reshape(lead + (4, 8))


def hybrid_encode(state: dict, flags: int, codec: int) -> dict:
    """The paper's export (Sec. 3.4): F_uv and every F_uvt slice reconstructed from the
    trained state as training with `flags` reads it, quantised to 8 bits and block-encoded
    in `codec` (encode_map); planes rounded to 8 bits (rint of the float32 product 255 v);
    the decoder as trained."""
    d = state["dims"]
    sc = d.get("codec", 0)
    fuv = encode_map(_map_texels_u8(state["fuv_ep"], state["fuv_w"], flags, sc), codec)
    fuvt = encode_map(_map_texels_u8(state["fuvt_ep"], state["fuvt_w"], flags, sc), codec)
    q = lambda a: np.rint(np.float32(255.0) * np.asarray(a, dtype=np.float32)).astype(np.uint8)
    return dict(W=d["W"], H=d["H"], Gu=d["Gu"], Gv=d["Gv"], S=d["S"], U=d["U"], V=d["V"], Tt=d["Tt"],
                hidden=d["hidden"], codec=codec, fuv=fuv, fuvt=fuvt, fut=q(state["fut"]), fvt=q(state["fvt"]),
                keys=np.asarray(d["keys"], dtype=np.float32), mlp=np.asarray(state["mlp"], dtype=np.float32))


def _decode_map(blocks, codec: int, lead: tuple, H: int, W: int) -> np.ndarray:
    """8-bit texels [..][H][W][4] of a block-compressed map."""
    ys, xs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    blocks = np.asarray(blocks, dtype=np.uint8)
    out = []
    for idx in np.ndindex(*lead):
        b = blocks[idx]
        sel = b[ys >> 2, xs >> 2]
        out.append(bc7_texels(sel, xs, ys) if codec == 1 else bc4_texels(sel, xs, ys))
    return np.stack(out).reshape(lead + (H, W, 4))


def hybrid_import(model: dict, frames: int) -> dict:
    """A directly parameterised training state (codec 0 layout, flag DIRECT) holding a
    compressed model: F_uv / F_uvt weights = decoded byte / 255 (float32 division), endpoints
    (0, 1) (so the plain Eq. (7) lerp reads the same values), planes = byte / 255, the decoder
    in float32.  Fine-tuning the decoder on it with frozen features (DIRECT | QPLANES) trains
    on exactly what a decode of the model reads (Sec. 4, final training stage)."""
    codec = model.get("codec", 0)
    H, W, S, Gu, Gv = model["H"], model["W"], model["S"], model["Gu"], model["Gv"]
    f32 = lambda q: np.asarray(q, dtype=np.float32) / np.float32(255.0)
    uv = _decode_map(model["fuv"], codec, (), H, W)
    uvt = _decode_map(model["fuvt"], codec, (S,), Gv, Gu)
    ep = lambda lead: np.stack([np.zeros(lead + (4,), np.float32), np.ones(lead + (4,), np.float32)], axis=-1)
    dims = dict(W=W, H=H, Gu=Gu, Gv=Gv, S=S, U=model["U"], V=model["V"], Tt=model["Tt"], hidden=model["hidden"],
                frames=frames, keys=np.asarray(model.get("keys", []), dtype=np.float32), codec=0)
    return dict(dims=dims, fuv_ep=ep((H // 4, W // 4)), fuv_w=f32(uv), fuvt_ep=ep((S, Gv // 4, Gu // 4)),
                fuvt_w=f32(uvt), fut=f32(model["fut"]), fvt=f32(model["fvt"]),
                mlp=np.asarray(model["mlp"], dtype=np.float32).copy())


# --------------------------------------------------------------------------------------
# Evaluation: tiled PSNR (supplementary Sec. D.2) and bit-rate (Tables 2-3)
# --------------------------------------------------------------------------------------

def psnr_tiled(pred: np.ndarray, target: np.ndarray, tile: int = 128):
    """Mean of per-tile PSNR over all tiles of all maps, and a global PSNR.

    ``pred``/``target`` are [T][H][W][3].  Per tile the peak is (max - min) of the
    target over the tile's texels and channels; PSNR = 10 log10(range^2 / MSE).
    Reading: a tile of zero range is skipped, a tile with MSE = 0 scores 100 dB.  All
    texels are valid (synthetic data has no mask).  Global PSNR uses the range and MSE
    over everything.
    """
    p = np.asarray(pred, dtype=np.float64)
    g = np.asarray(target, dtype=np.float64)
    T, H, W, _ = g.shape
    scores = []
    for k in range(T):
        for y0 in range(0, H, tile):
            for x0 in range(0, W, tile):
                gt = g[k, y0:y0 + tile, x0:x0 + tile]
                pr = p[k, y0:y0 + tile, x0:x0 + tile]
                rng = gt.max() - gt.min()
                if rng <= 0:
                    continue
                mse = np.mean((pr - gt) ** 2)
                scores.append(100.0 if mse == 0 else 10.0 * np.log10(rng * rng / mse))
    mse_all = np.mean((p - g) ** 2)
    rng_all = g.max() - g.min()
    glob = 100.0 if mse_all == 0 else 10.0 * np.log10(rng_all * rng_all / mse_all)
    return (float(np.mean(scores)) if scores else float("nan")), float(glob)


def bits_per_texel_paper(W: int, H: int, n_maps: int, uvt_res: tuple, hidden: int,
                         uv_ch=4, plane_len=64, plane_t=24, plane_ch=2) -> float:
    """Bits per texel per map of the paper's hybrid layout (Table 1, Table 3).

    F_uv (W x H, 4 channels) and each time slice of F_uvt are BC7 at 8 bits per texel;
    F_ut and F_vt (plane_len x plane_t x 2 channels) are 8-bit; the MLP 16-h-h-3 is
    FP16.  Divided by W * H * n_maps.
    """
    uw, uh, ut = uvt_res
    bits = W * H * 8                       # F_uv, BC7
    bits += uw * uh * ut * 8               # F_uvt slices, BC7
    bits += 2 * plane_len * plane_t * plane_ch * 8
    n_in = 16
    params = hidden * n_in + hidden + hidden * hidden + hidden + 3 * hidden + 3
    bits += params * 16
    return bits / (W * H * n_maps)


def bits_per_texel_bc4_grid(W: int, H: int, Gw: int, Gh: int, T: int,
                            grid_bits=16, mlp_bits=16) -> float:
    """Bits per texel per key of the 8-channel BC4 map + 8-channel grid + MLP layout.

    BC4 stores 8 bytes per 4x4 block per channel (4 bits per texel per channel).
    """
    bits = W * H * N_SPATIAL * 4
    bits += Gw * Gh * T * N_GRID * grid_bits
    bits += MLP_SIZE * mlp_bits
    return bits / (W * H * T)
