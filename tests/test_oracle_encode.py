"""Pins for the oracle's texel-value block encoders and the paper's export path (Sec. 3.4:
reconstruct the trained maps, quantise to 8 bits, block-compress; supplementary ablation:
the "w/o BC simulation" arm optimises the maps directly).  Each test checks the oracle
against something other than itself: brute-force searches written here from the format
definitions, blocks that a block of the format reproduces exactly, closed-form tie cases,
finite differences, and the pinned decoders and exact exports."""
import numpy as np

from oracle import ndgi_oracle as O
from paper_2604_12625_amd import inputs as I

W4 = (0, 4, 9, 13, 17, 21, 26, 30, 34, 38, 43, 47, 51, 55, 60, 64)   # BC7's 4-bit weight table


# ------------------------------------------------------------------------------ BC4
def _all_palettes_scalar():
    """[65536][8] palettes from the scalar (separately pinned) palette function."""
    return np.array([O.bc4_palette(p >> 8, p & 255) for p in range(65536)], dtype=np.int64)


def test_bc4_encoder_is_the_exhaustive_optimum():
    pal = _all_palettes_scalar()
    g = np.random.default_rng(11)
    blocks = [g.integers(0, 256, 16), g.integers(90, 110, 16), np.r_[np.zeros(8, int), np.full(8, 255)],
              np.clip(np.round(np.linspace(30, 200, 16) + g.normal(0, 6, 16)), 0, 255).astype(int)]
    for X in blocks:
        enc = O.encode_bc4(X[None])[0]
        dec = O.bc4_decode_block(enc).reshape(16).astype(np.int64)
        sse = int(((dec - X) ** 2).sum())
        best = int(((pal[:, None, :] - X[None, :, None]) ** 2).min(-1).sum(-1).min())
        assert sse == best, (sse, best)


def test_bc4_encoder_reproduces_every_decodable_block():
    g = np.random.default_rng(12)
    blocks = g.integers(0, 256, (60, 8)).astype(np.uint8)
    blocks[:30, 0] = np.maximum(blocks[:30, 0], blocks[:30, 1] + 1)      # 8-value mode
    blocks[30:, 0] = np.minimum(blocks[30:, 0], blocks[30:, 1])          # 6-value mode
    tex = O.bc4_decode_blocks(blocks)
    np.testing.assert_array_equal(O.bc4_decode_blocks(O.encode_bc4(tex)), tex)


def test_bc4_encoder_tie_rule_on_a_constant_block():
    # 100 in every texel: no pair below e0 * 256 + e1 = 100 reaches it (e0 = 0 needs e1 >= 100
    # in the 6-value palette), and (0, 100) does through selector 1 (e1)
    enc = O.encode_bc4(np.full((1, 16), 100))[0]
    assert enc[0] == 0 and enc[1] == 100
    assert (O.bc4_codes(enc) == 1).all()
    # 255 everywhere: pair (0, 0) through the constant selector 7
    enc = O.encode_bc4(np.full((1, 16), 255))[0]
    assert enc[0] == 0 and enc[1] == 0 and (O.bc4_codes(enc) == 7).all()


# ------------------------------------------------------------------------------ BC7 mode 6
def _fields(block):
    """(E0 [4], E1 [4], idx [16]) of a mode-6 block, from the format definition."""
    b = int.from_bytes(bytes(block), "little")
    assert b & 0x7F == 0x40
    v = [(b >> (7 + 7 * k)) & 0x7F for k in range(8)]
    p0, p1 = (b >> 63) & 1, (b >> 64) & 1
    idx = [(b >> 65) & 7] + [(b >> (64 + 4 * i)) & 0xF for i in range(1, 16)]
    return [2 * v[2 * c] + p0 for c in range(4)], [2 * v[2 * c + 1] + p1 for c in range(4)], idx


def _texel(E0, E1, j):
    return np.array([((64 - W4[j]) * E0[c] + W4[j] * E1[c] + 32) >> 6 for c in range(4)])


def _best_sse(E0, E1, X):
    """Least summed squared error over free per-texel indices (brute force over 16)."""
    pal = np.stack([_texel(E0, E1, j) for j in range(16)])           # [16][4]
    return int(((pal[None] - X[:, None]) ** 2).sum(-1).min(-1).sum())


def _smooth_blocks(g, n, noise):
    e1, e2, w = g.uniform(0, 255, (n, 1, 4)), g.uniform(0, 255, (n, 1, 4)), g.uniform(0, 1, (n, 16, 1))
    return np.clip(np.rint((1 - w) * e1 + w * e2 + g.normal(0, noise, (n, 16, 4))), 0, 255).astype(np.int64)


def _test_blocks(seed):
    g = np.random.default_rng(seed)
    return np.concatenate([g.integers(0, 256, (12, 16, 4)), _smooth_blocks(g, 12, 0.0), _smooth_blocks(g, 12, 5.0),
                           np.repeat(g.integers(0, 256, (6, 16, 1)), 4, axis=2)])


def test_bc7_encoder_recovers_blocks_that_use_both_end_indices():
    g = np.random.default_rng(13)
    blocks = I.random_bc7m6((80,), g)
    tex = []
    for b in blocks:
        bits = int.from_bytes(bytes(b), "little")
        bits &= ~(7 << 65)                           # texel 0: index 0
        s = 1 + int(g.integers(0, 15))
        bits |= 0xF << (64 + 4 * s)                  # another texel: index 15
        tex.append(O.bc7m6_decode_block(np.frombuffer(bits.to_bytes(16, "little"), np.uint8)))
    tex = np.stack(tex).astype(np.int64)
    enc = O.encode_bc7m6(tex)
    np.testing.assert_array_equal(np.stack([O.bc7m6_decode_block(b) for b in enc]), tex)


def test_bc7_encoder_anchor_mode_bits_and_optimal_indices():
    X = _test_blocks(14)
    for b, x in zip(O.encode_bc7m6(X), X):
        E0, E1, idx = _fields(b)
        assert idx[0] < 8
        for s in range(16):
            errs = [int(((_texel(E0, E1, j) - x[s]) ** 2).sum()) for j in range(16)]
            assert errs[idx[s]] == min(errs), (s, idx[s], errs)


def test_bc7_encoder_ends_in_a_local_minimum_of_its_moves():
    """No single move of the final search step (a 7-bit endpoint value +-1, all four values of
    one endpoint +-1, a p-bit flipped) with refitted indices is strictly better."""
    X = _test_blocks(15)
    for b, x in zip(O.encode_bc7m6(X), X):
        E0, E1, _ = _fields(b)
        ends = [[E0[c] >> 1 for c in range(4)], [E1[c] >> 1 for c in range(4)]]
        ps = [E0[0] & 1, E1[0] & 1]
        cur = _best_sse(E0, E1, x)

        def sse_of(v, p):
            return _best_sse([2 * v[0][c] + p[0] for c in range(4)], [2 * v[1][c] + p[1] for c in range(4)], x)
        for k in range(2):
            for d in (-1, 1):
                for c in list(range(4)) + [None]:
                    v = [list(ends[0]), list(ends[1])]
                    cols = range(4) if c is None else [c]
                    for cc in cols:
                        v[k][cc] += d
                    if all(0 <= v[k][cc] <= 127 for cc in cols):
                        assert sse_of(v, ps) >= cur
            p = list(ps)
            p[k] ^= 1
            assert sse_of([ends[0], ends[1]], p) >= cur


def test_bc7_encoder_on_grey_blocks_against_the_exhaustive_optimum():
    """Grey blocks (equal channels): the four channels pose the same problem with shared
    indices and p-bits, so some optimum has grey endpoints, and every 8-bit grey endpoint is
    a mode-6 endpoint ((E >> 1) << 1 | (E & 1)); all 65536 grey pairs are searched here.
    The encoder is not exhaustive: it never beats the optimum, reaches it on most smooth
    blocks, and stays within the stated mean excess."""
    g = np.random.default_rng(16)
    E = np.arange(256)
    w = np.asarray(W4)
    pal = ((64 - w)[None, None, :] * E[:, None, None] + w[None, None, :] * E[None, :, None] + 32) >> 6
    rows = []
    for i in range(32):
        if i % 2 == 0:
            gv = np.clip(np.round(np.linspace(g.integers(0, 128), g.integers(128, 256), 16) + g.normal(0, 3, 16)), 0, 255)
        else:
            gv = g.integers(0, 256, 16)
        gv = gv.astype(np.int64)
        opt = 4 * int(((pal[:, :, None, :] - gv[None, None, :, None]) ** 2).min(-1).sum(-1).min())
        X = np.repeat(gv[:, None], 4, axis=1)
        dec = O.bc7m6_decode_block(O.encode_bc7m6(X[None])[0]).astype(np.int64)
        rows.append((int(((dec - X) ** 2).sum()), opt))
    enc, opt = np.array(rows).T
    assert (enc >= opt).all()
    # measured on this set: the optimum in about half of the blocks, a mean excess of about
    # 6% of the optimum's error
    assert np.mean(enc == opt) >= 0.3, rows
    assert np.mean(enc - opt) <= 0.12 * np.mean(opt), rows


# ------------------------------------------------------------------------------ hybrid export path
def _tiny(codec, seed, hidden=16):
    g = np.random.default_rng(seed)
    keys = np.sort(g.uniform(0, 1, 3)).astype(np.float32)
    st = I.hybrid_train_init(8, 8, "L", 3, keys, g, slices=3, plane=(4, 4, 3), codec=codec)
    st["dims"].update(Gu=4, Gv=4)
    cw = () if codec else (4,)
    st["fuvt_ep"] = st["fuvt_ep"][:, :1, :1]
    st["fuvt_w"] = g.uniform(0, 1, (3, 4, 4) + cw).astype(np.float32)
    return st


def test_encode_under_simulation_equals_the_exact_export():
    """With BCSIM the reconstructed texels are those of the exact export, which a block of the
    format reproduces: the encoder's blocks decode to the export's decode (BC4 exhaustive; the
    BC7 blocks here use index 0 and 15 in every footprint)."""
    for codec in (0, 1):
        st = _tiny(codec, 21 + codec)
        if codec:
            for k in ("fuv_w", "fuvt_w"):          # texel (0, 0) and (1, 1) of every footprint
                a = st[k]
                a[..., 0::4, 0::4] = 0.0
                a[..., 1::4, 1::4] = 1.0
        ex, en = O.hybrid_export(st), O.hybrid_encode(st, O.HT_BCSIM, codec)
        for key, lead, H, W in (("fuv", (), 8, 8), ("fuvt", (3,), 4, 4)):
            np.testing.assert_array_equal(O._decode_map(en[key], codec, lead, H, W),
                                          O._decode_map(ex[key], codec, lead, H, W))
        np.testing.assert_array_equal(en["fut"], ex["fut"])


def test_plain_and_direct_reconstruction_closed_forms():
    st = _tiny(0, 30)
    # endpoints (0, 1): the float32 lerp is the weight itself, and DIRECT reads the weight
    st["fuv_ep"][..., 0], st["fuv_ep"][..., 1] = 0.0, 1.0
    q = np.clip(np.rint(np.float32(255) * st["fuv_w"].astype(np.float32)), 0, 255)
    np.testing.assert_array_equal(O._map_texels_u8(st["fuv_ep"], st["fuv_w"], 0, 0), q)
    np.testing.assert_array_equal(O._map_texels_u8(st["fuv_ep"] * 0 + 0.3, st["fuv_w"], O.HT_DIRECT, 0), q)
    # equal endpoints: every texel is the endpoint whatever the weight
    st["fuv_ep"][..., 1] = st["fuv_ep"][..., 0] = 0.6
    np.testing.assert_array_equal(O._map_texels_u8(st["fuv_ep"], st["fuv_w"], 0, 0), np.rint(np.float32(255) * np.float32(0.6)))


def test_import_is_read_back_by_the_direct_forward_as_the_decode():
    for codec in (0, 1):
        m = I.random_hybrid_model(W=16, H=12, profile="L", slices=3, plane=(8, 6, 4), keys=True, config=31 + codec,
                                  codec=codec, uvt_side=(4, 4))
        m["mlp"] = np.asarray(m["mlp"], np.float32)
        st = O.hybrid_import(m, frames=len(m["keys"]))
        d = st["dims"]
        y, x = np.meshgrid(np.arange(d["H"]), np.arange(d["W"]), indexing="ij")
        for f in range(d["frames"]):
            n = x.size
            fwd = O.hybrid_train_forward(st, x.ravel(), y.ravel(), np.full(n, f), O.HT_DIRECT | O.HT_QPLANES)
            t = np.full(n, np.float64(d["keys"][f]))
            dec = O.hybrid_decode_f64(m, (x.ravel() + 0.5) / d["W"], (y.ravel() + 0.5) / d["H"], t)
            np.testing.assert_allclose(fwd, dec, rtol=0, atol=1e-6 * np.abs(dec).max())
        # and the exhaustive BC4 encoder gives the imported texels back exactly
        if codec == 0:
            en = O.hybrid_encode(st, O.HT_DIRECT, 0)
            np.testing.assert_array_equal(O._decode_map(en["fuv"], 0, (), 12, 16), O._decode_map(m["fuv"], 0, (), 12, 16))


def test_direct_gradients_match_finite_differences():
    from test_oracle_hybrid import _batch, _fd_check, tiny_hybrid_state
    st = tiny_hybrid_state(16, seed=40)
    xs, ys, fs, tgt = _batch(st, 40, seed=41)
    _fd_check(st, xs, ys, fs, tgt, O.HT_DIRECT | O.HT_NOISE, O.HYB_KEYS)
    _, g = O.hybrid_train_grads(st, xs, ys, fs, tgt, O.HT_DIRECT)
    assert not g["fuv_ep"].any() and not g["fuvt_ep"].any()


# --------------------------------------------------------------- BC7 modes 4, 5 and 6
def _pillow_bc7(blocks):
    """[n][16][4] texels of BC7 blocks [n][16] decoded by Pillow's BC7 decoder (a DDS file in
    memory, DXGI_FORMAT_BC7_UNORM): a decoder independent of the oracle."""
    import io
    import struct
    import pytest
    Image = pytest.importorskip("PIL.Image")
    blocks = np.asarray(blocks, dtype=np.uint8).reshape(-1, 16)
    n = blocks.shape[0]
    wb = 1
    while wb * wb < n:
        wb *= 2
    hb = (n + wb - 1) // wb
    data = np.zeros((wb * hb, 16), np.uint8)
    data[:n] = blocks
    hdr = struct.pack("<4sI", b"DDS ", 124)
    hdr += struct.pack("<IIIIII", 0x1 | 0x2 | 0x4 | 0x1000 | 0x80000, 4 * hb, 4 * wb, wb * hb * 16, 0, 1) + b"\0" * 44
    hdr += struct.pack("<II4sIIIII", 32, 0x4, b"DX10", 0, 0, 0, 0, 0)
    hdr += struct.pack("<IIIII", 0x1000, 0, 0, 0, 0)
    hdr += struct.pack("<IIIII", 98, 3, 0, 1, 0)
    img = Image.open(io.BytesIO(hdr + data.tobytes()))
    img.load()
    px = np.asarray(img.convert("RGBA")).reshape(hb, 4, wb, 4, 4).transpose(0, 2, 1, 3, 4).reshape(-1, 16, 4)
    return px[:n]


def test_bc7_decoder_modes_4_5_6_match_pillow():
    blocks = I.random_bc7((3000,), np.random.default_rng(31))
    ref = _pillow_bc7(blocks)
    np.testing.assert_array_equal(np.stack([O.bc7_decode_block(b) for b in blocks]), ref)
    xs, ys = np.tile(np.arange(4), 4), np.repeat(np.arange(4), 4)
    np.testing.assert_array_equal(O.bc7_texels(np.repeat(blocks[:, None], 16, 1), xs[None], ys[None]), ref)
    assert set(O.bc7_mode(b) for b in blocks) == {4, 5, 6}


def _end_index_blocks(g, n):
    """Random mode 4 / 5 / 6 blocks whose every index set uses its lowest index at texel 0
    and its highest at texel 15 (so texels 0 and 15 are the endpoints of each set)."""
    out = I.random_bc7((n,), g)
    for blk in out:
        b = int.from_bytes(bytes(blk), "little")
        m = O.bc7_mode(blk)
        sets = {6: ((65, 4),), 5: ((66, 2), (97, 2)), 4: ((50, 2), (81, 3))}[m]
        for pos, bits in sets:
            b &= ~(((1 << (bits - 1)) - 1) << pos)                 # texel 0: index 0
            last = pos + bits - 1 + bits * 14
            b |= ((1 << bits) - 1) << last                        # texel 15: the top index
        blk[:] = np.frombuffer(b.to_bytes(16, "little"), np.uint8)
    return out


def test_bc7_multimode_encoder_reproduces_blocks_using_both_end_indices():
    blocks = _end_index_blocks(np.random.default_rng(32), 48)
    tex = np.stack([O.bc7_decode_block(b) for b in blocks])
    enc = O.encode_bc7(tex)
    np.testing.assert_array_equal(_pillow_bc7(enc), tex)


def test_bc7_multimode_encoder_is_valid_and_never_worse_than_mode_6():
    g = np.random.default_rng(33)
    tex = np.concatenate([g.integers(0, 256, (30, 16, 4)), _smooth_blocks(g, 30, 8)]).astype(np.uint8)
    enc = O.encode_bc7(tex)
    assert set(O.bc7_mode(b) for b in enc) <= {4, 5, 6}
    got = _pillow_bc7(enc).astype(np.int64)
    sse = ((got - tex) ** 2).sum((1, 2))
    sse6 = ((_pillow_bc7(O.encode_bc7m6(tex)).astype(np.int64) - tex) ** 2).sum((1, 2))
    assert (sse <= sse6).all()
    assert sse.sum() < sse6.sum()            # the other modes win on some of these blocks


def test_bc7_subset_search_ends_in_a_local_minimum_of_its_moves():
    """For each precision of modes 4 and 5, no single move of the search (one value +-1, all
    values +-1) lowers the error of its result, checked by brute force on the moves."""
    g = np.random.default_rng(34)
    for (n, b, C) in ((7, 2, 3), (8, 2, 1), (5, 2, 3), (5, 3, 3), (6, 3, 1), (6, 2, 1)):
        X = g.integers(0, 256, (6, 16, C))
        v0, v1, J, sse = O._sub_search(X, n, b)
        Wt = np.asarray({2: (0, 21, 43, 64), 3: (0, 9, 18, 27, 37, 46, 55, 64)}[b])
        top = (1 << n) - 1

        def err(a, z, x):
            ea = (a << (8 - n)) | (a >> (2 * n - 8)) if n < 8 else a
            ez = (z << (8 - n)) | (z >> (2 * n - 8)) if n < 8 else z
            pal = ((64 - Wt)[:, None] * ea[None] + Wt[:, None] * ez[None] + 32) >> 6   # [index][C]
            return int(((pal[None] - x[:, None]) ** 2).sum(-1).min(-1).sum())
        for i in range(6):
            assert err(v0[i], v1[i], X[i]) == sse[i]
            for k in (0, 1):
                for c in list(range(C)) + ([C] if C > 1 else []):
                    for dv in (-1, 1):
                        a, z = v0[i].copy(), v1[i].copy()
                        v = a if k == 0 else z
                        if c == C:
                            v += dv
                        else:
                            v[c] += dv
                        if (v < 0).any() or (v > top).any():
                            continue
                        assert err(a, z, X[i]) >= sse[i], (n, b, C, i, k, c, dv)
