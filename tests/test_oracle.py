"""Pins for the CPU reference: each test checks the oracle against something other than
itself -- values worked out by hand from the paper's equations (tests/golden), closed
forms, exact reproduction properties, finite differences, or an independent library
routine (torch.optim.Adam)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import ndgi_oracle as O
from paper_2604_12625_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_blocks():
    rows = []
    for line in open(os.path.join(GOLDEN, "bc4_blocks.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        a, b = line.split("|")
        rows.append((np.array([int(h, 16) for h in a.split()], dtype=np.uint8),
                     np.array([int(v) for v in b.split()], dtype=np.uint8)))
    return rows


# ---------------------------------------------------------------- block compression

def test_bc4_golden_blocks():
    rows = _golden_blocks()
    assert len(rows) == 7
    for blk, want in rows:
        np.testing.assert_array_equal(O.bc4_decode_block(blk).ravel(), want)
        np.testing.assert_array_equal(O.bc4_decode_blocks(blk[None])[0], want)


def test_bc4_palette_exhaustive_integer_rounding():
    # Round-to-nearest of N/D written as (2N + D) // (2D): a different formulation from the
    # oracle's floor((N + (D-1)/2) / D); covers all 65536 endpoint pairs and all codes.
    e0, e1 = np.meshgrid(np.arange(256), np.arange(256), indexing="ij")
    e0 = e0.ravel()
    e1 = e1.ravel()
    for code in range(8):
        c = np.full_like(e0, code)
        got = O.bc4_palette_value(e0, e1, c).astype(np.int64)
        if code == 0:
            want = e0
        elif code == 1:
            want = e1
        else:
            j = code - 1
            want8 = (2 * ((7 - j) * e0 + j * e1) + 7) // 14
            if code <= 5:
                want6 = (2 * ((5 - j) * e0 + j * e1) + 5) // 10
            else:
                want6 = np.full_like(e0, 0 if code == 6 else 255)
            want = np.where(e0 > e1, want8, want6)
        np.testing.assert_array_equal(got, want)


def test_bc4_palette_vs_exact_rationals():
    # Eq. (7): (1 - w) e_a + w e_b with w = j/7 or j/5, as exact fractions, rounded.
    g = np.random.default_rng(1)
    pairs = g.integers(0, 256, size=(3000, 2))
    pairs = np.concatenate([pairs, [[0, 0], [255, 255], [255, 0], [0, 255], [1, 0], [0, 1]]])
    for e0, e1 in pairs:
        pal = O.bc4_palette(e0, e1)
        if e0 > e1:
            ws = [Fraction(0), Fraction(1)] + [Fraction(j, 7) for j in range(1, 7)]
            exact = [(1 - w) * int(e0) + w * int(e1) for w in ws]
        else:
            ws = [Fraction(0), Fraction(1)] + [Fraction(j, 5) for j in range(1, 5)]
            exact = [(1 - w) * int(e0) + w * int(e1) for w in ws] + [Fraction(0), Fraction(255)]
        assert pal == [int(round(x)) for x in exact]


def test_bc4_vectorised_matches_scalar_on_random_blocks():
    g = np.random.default_rng(2)
    blocks = g.integers(0, 256, size=(500, 8), dtype=np.uint8)
    want = np.stack([O.bc4_decode_block(b).ravel() for b in blocks])
    np.testing.assert_array_equal(O.bc4_decode_blocks(blocks), want)


# ------------------------------------------------------------------ interpolation

def identity_mlp(sel=(0, 1, 8), b1=None):
    """App. identity decoder: W1 = [I16; 0], W2 = I32, W3 selects features -> rgb = exp(x_sel)."""
    p = np.zeros(O.MLP_SIZE)
    W1 = np.zeros((32, 16))
    W1[:16, :16] = np.eye(16)
    W2 = np.eye(32)
    W3 = np.zeros((3, 32))
    for r, c in enumerate(sel):
        W3[r, c] = 1.0
    p[O.MLP_W1:O.MLP_B1] = W1.ravel()
    if b1 is not None:
        p[O.MLP_B1:O.MLP_W2] = b1
    p[O.MLP_W2:O.MLP_B2] = W2.ravel()
    p[O.MLP_W3:O.MLP_B3] = W3.ravel()
    return p


def small_model(W=64, H=64, Gw=16, Gh=16, T=8, seed=0):
    m = I.random_model(W, H, Gw, Gh, T, config=99, index=seed)
    m["grid"] = np.abs(m["grid"])            # non-negative so ReLU passes G unchanged
    m["mlp"] = identity_mlp()
    return m


def test_texel_centres_return_stored_texels():
    m = small_model()
    W, H = m["W"], m["H"]
    q = I.texel_centre_queries(W, H, [0.3])
    rgb = O.decode(m, q)
    x = np.tile(np.arange(W), H)
    y = np.repeat(np.arange(H), W)
    dec = O.bc4_decode_blocks(m["bc4"].reshape(-1, 8)).reshape(H // 4, W // 4, 8, 16)
    want0 = dec[y >> 2, x >> 2, 0, 4 * (y & 3) + (x & 3)] / 255.0
    want1 = dec[y >> 2, x >> 2, 1, 4 * (y & 3) + (x & 3)] / 255.0
    np.testing.assert_allclose(np.log(rgb[:, 0]), want0, rtol=0, atol=1e-14)
    np.testing.assert_allclose(np.log(rgb[:, 1]), want1, rtol=0, atol=1e-14)


def _affine_bc4(W, H, c0=10):
    """BC4 map whose channel-0 texels equal x + y + c0 (8-value blocks e0 = b+7, e1 = b)."""
    bc4 = np.zeros((H // 4, W // 4, 8, 8), dtype=np.uint8)
    for by in range(H // 4):
        for bx in range(W // 4):
            base = 4 * bx + 4 * by + c0
            field = 0
            for s in range(16):
                d = (s % 4) + (s // 4)                 # (x%4) + (y%4)
                code = 1 if d == 0 else 8 - d          # value = base + 7 - j, j = code - 1
                field |= code << (3 * s)
            blk = [base + 7, base] + [(field >> (8 * k)) & 0xFF for k in range(6)]
            bc4[by, bx, :, :] = np.array(blk, dtype=np.uint8)
    return bc4


def test_spatial_bilinear_reproduces_affine_field():
    m = small_model()
    W, H = m["W"], m["H"]
    m["bc4"] = _affine_bc4(W, H)
    # sanity of the construction against the pinned codec
    dec = O.bc4_decode_blocks(m["bc4"].reshape(-1, 8)).reshape(H // 4, W // 4, 8, 16)
    assert dec[3, 5, 0, 4 * 2 + 1] == (4 * 5 + 1) + (4 * 3 + 2) + 10
    g = np.random.default_rng(3)
    u = g.uniform(1.0 / W, 1 - 1.0 / W, 2000)
    v = g.uniform(1.0 / H, 1 - 1.0 / H, 2000)
    rgb = O.decode_f64(m, u, v, np.full_like(u, 0.1))
    S0 = np.log(rgb[:, 0]) * 255.0
    np.testing.assert_allclose(S0, (u * W - 0.5) + (v * H - 0.5) + 10, rtol=0, atol=1e-9)


def test_grid_reproduces_affine_field_in_space_and_time():
    W, H, Gw, Gh, T = 64, 64, 16, 16, 8
    m = small_model(W, H, Gw, Gh, T)
    k, gy, gx = np.meshgrid(np.arange(T), np.arange(Gh), np.arange(Gw), indexing="ij")
    m["grid"] = np.zeros((T, Gh, Gw, 8))
    m["grid"][..., 0] = 0.05 * gx + 0.03 * gy + 0.11 * k + 0.2
    g = np.random.default_rng(4)
    u = g.uniform(1.0 / Gw, 1 - 1.0 / Gw, 2000)
    v = g.uniform(1.0 / Gh, 1 - 1.0 / Gh, 2000)
    t = g.uniform(0.0, (T - 1) / T, 2000)              # no wrap between last key and key 0
    rgb = O.decode_f64(m, u, v, t)
    G0 = np.log(rgb[:, 2])
    want = 0.05 * (u * Gw - 0.5) + 0.03 * (v * Gh - 0.5) + 0.11 * (t * T) + 0.2
    np.testing.assert_allclose(G0, want, rtol=0, atol=1e-12)


def test_grid_node_values_at_node_centres_and_keys():
    W, H, Gw, Gh, T = 64, 64, 16, 16, 8
    m = small_model(W, H, Gw, Gh, T)
    g = np.random.default_rng(5)
    kk = g.integers(0, T, 300)
    yy = g.integers(0, Gh, 300)
    xx = g.integers(0, Gw, 300)
    rgb = O.decode_f64(m, (xx + 0.5) / Gw, (yy + 0.5) / Gh, kk / T)
    np.testing.assert_allclose(np.log(rgb[:, 2]), m["grid"][kk, yy, xx, 0], rtol=0, atol=1e-7)


def test_time_is_periodic_and_wraps_last_key_to_first():
    W, H, Gw, Gh, T = 64, 64, 16, 16, 8
    m = small_model(W, H, Gw, Gh, T)
    g = np.random.default_rng(6)
    u, v, t = g.random(500), g.random(500), g.random(500)
    a = O.decode_f64(m, u, v, t)
    b = O.decode_f64(m, u, v, t + 1.0)
    c = O.decode_f64(m, u, v, t - 3.0)
    np.testing.assert_allclose(a, b, rtol=1e-12)
    np.testing.assert_allclose(a, c, rtol=1e-12)
    # halfway between the last key (T-1) and key 0 of the next day
    gx, gy = 3, 5
    rgb = O.decode_f64(m, np.array([(gx + 0.5) / Gw]), np.array([(gy + 0.5) / Gh]),
                       np.array([(T - 0.5) / T]))
    want = 0.5 * (m["grid"][T - 1, gy, gx, 0] + m["grid"][0, gy, gx, 0])
    np.testing.assert_allclose(np.log(rgb[0, 2]), want, atol=1e-7)


def test_clamp_to_edge_outside_unit_square():
    m = small_model()
    q = np.array([[-0.5, 0.5, 0.2], [1.7, 0.5, 0.2], [0.5, -3.0, 0.2], [0.5, 9.0, 0.2]], dtype=np.float32)
    e = np.array([[0.0, 0.5, 0.2], [0.9999, 0.5, 0.2], [0.5, 0.0, 0.2], [0.5, 0.9999, 0.2]], dtype=np.float32)
    np.testing.assert_allclose(O.decode(m, q), O.decode(m, e), rtol=1e-12)


def test_non_finite_queries_decode_to_nan():
    m = small_model()
    q = np.array([[np.nan, 0.5, 0.2], [0.5, np.inf, 0.2], [0.5, 0.5, -np.inf], [0.5, 0.5, 0.5]],
                 dtype=np.float32)
    out = O.decode(m, q)
    assert np.isnan(out[:3]).all() and np.isfinite(out[3]).all()


# ------------------------------------------------------------------------- decoder MLP

def test_mlp_identity_bias_and_relu():
    m = small_model()
    m["grid"] = -np.abs(m["grid"]) - 0.1            # G0 < 0 -> ReLU gives exp(0) = 1
    q = I.uniform_queries(300, np.random.default_rng(7))
    base = O.decode(m, q)
    np.testing.assert_array_equal(base[:, 2], 1.0)
    b1 = np.zeros(32)
    b1[0] = 0.25
    b1[1] = -10.0
    m["mlp"] = identity_mlp(b1=b1)
    out = O.decode(m, q)
    np.testing.assert_allclose(np.log(out[:, 0]), np.log(base[:, 0]) + 0.25, atol=1e-13)
    np.testing.assert_array_equal(out[:, 1], 1.0)   # S1 - 10 < 0 -> ReLU -> 0


def test_mlp_layer_orientation_with_permutation():
    # W2 a non-symmetric permutation: output r reads hidden unit perm[sel[r]]; a transposed
    # W2 would read the inverse permutation instead.
    m = small_model()
    perm = np.roll(np.arange(32), -5)             # perm[i] = (i + 5) % 32
    p = identity_mlp(sel=(3, 4, 7))
    W2 = np.zeros((32, 32))
    W2[np.arange(32), perm] = 1.0                  # h2[i] = h1[perm[i]]
    p[O.MLP_W2:O.MLP_B2] = W2.ravel()
    m["mlp"] = p
    q = I.uniform_queries(200, np.random.default_rng(8))
    x = O.features(m, q[:, 0].astype(np.float64), q[:, 1].astype(np.float64), q[:, 2].astype(np.float64))
    out = np.log(O.decode(m, q))
    np.testing.assert_allclose(out, np.maximum(0, x[:, perm[[3, 4, 7]]]), atol=1e-13)


def test_page_decode_equals_texel_centre_queries():
    m = I.random_model(256, 256, 64, 64, 24, np.float16, np.float16, config=98)
    t = np.float32(0.37)
    pg = O.decode_page(m, 1, 0, t, page=128)
    y, x = np.meshgrid(np.arange(128), 128 + np.arange(128), indexing="ij")
    q = np.stack([((x + 0.5) / 256).ravel(), ((y + 0.5) / 256).ravel(), np.full(128 * 128, t)], 1)
    np.testing.assert_allclose(pg.reshape(-1, 3), O.decode(m, q.astype(np.float32)), rtol=1e-13)
    dst = np.zeros((256 * 128, 3))
    bad = O.decode_pages([m], [(0, 1, 0, t, 128), (0, 2, 0, t, 0), (1, 0, 0, t, 0)], 128, dst, 256)
    assert bad == 2
    np.testing.assert_allclose(dst.reshape(128, 256, 3)[:, 128:], pg, rtol=0)


# ----------------------------------------------------------------------------- training

def tiny_state(seed=0, W=8, H=8, Gw=2, Gh=2, T=2):
    g = np.random.default_rng(seed)
    st = I.train_init(W, H, Gw, Gh, T, [0.5, 0.4, 0.3], g)
    st["grid"] = st["grid"] * 5.0
    return st


def _loss_with(state, xs, ys, ks, tgt, spatial_offset=None):
    if spatial_offset is None:
        return O.l2_loss(O.train_forward(state, xs, ys, ks), tgt)
    # forward with an additive offset on the spatial features of each texel
    d = state["dims"]
    val, *_ = O.bcsim_spatial(state["endpoints"], state["weights"], xs, ys)
    S = val / 255.0 + spatial_offset[ys, xs]
    grid = state["grid"].astype(np.float64)
    G = np.zeros_like(S)
    for (gy, gx, w) in O._sample_coords(d, xs, ys):
        G += w[:, None] * grid[ks, gy, gx]
    x = np.concatenate([S, G], 1)
    P = O.unpack_mlp(state["mlp"])
    h1 = np.maximum(0, x @ P["W1"].T + P["b1"])
    h2 = np.maximum(0, h1 @ P["W2"].T + P["b2"])
    return O.l2_loss(np.exp(h2 @ P["W3"].T + P["b3"]), tgt)


def test_loss_closed_form():
    st = tiny_state()
    xs, ys, ks = I.train_samples(64, 8, 8, 2, np.random.default_rng(1))
    rgb = O.train_forward(st, xs, ys, ks)
    assert abs(O.l2_loss(rgb, rgb + 0.125) - 0.015625) < 1e-15
    assert abs(O.l2_loss(rgb, rgb - 0.5) - 0.25) < 1e-15


def test_gradients_match_central_finite_differences():
    st = tiny_state(seed=3)
    st["grid"] = st["grid"].astype(np.float64)
    st["mlp"] = st["mlp"].astype(np.float64)
    g = np.random.default_rng(9)
    xs, ys, ks = I.train_samples(96, 8, 8, 2, g)
    tgt = g.uniform(0.2, 2.0, (96, 3))
    loss, gr = O.train_grads(st, xs, ys, ks, tgt)
    assert abs(loss - _loss_with(st, xs, ys, ks, tgt)) < 1e-15
    h = 1e-6
    for key in ("mlp", "grid"):
        flat = st[key].reshape(-1)
        idx = g.choice(flat.size, size=min(60, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = _loss_with(st, xs, ys, ks, tgt)
            flat[i] = old - h
            lm = _loss_with(st, xs, ys, ks, tgt)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = gr[key].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(fd)) + 1e-9, (key, i, fd, an)
    # spatial: FD w.r.t. an additive per-texel feature offset gives dL/df at each texel;
    # the straight-through factors (1 - J/7, J/7, (E2 - E1)/255) then map it to e1, e2, w.
    off = np.zeros((8, 8, 8))
    dLdf = np.zeros((8, 8, 8))
    for yy in range(8):
        for xx in range(8):
            for c in range(8):
                off[yy, xx, c] = h
                lp = _loss_with(st, xs, ys, ks, tgt, off)
                off[yy, xx, c] = -h
                lm = _loss_with(st, xs, ys, ks, tgt, off)
                off[yy, xx, c] = 0
                dLdf[yy, xx, c] = (lp - lm) / (2 * h)
    E1 = O.quantise_endpoint(st["endpoints"][..., 0])
    E2 = O.quantise_endpoint(st["endpoints"][..., 1])
    J = O.quantise_weight(st["weights"])
    want_w = dLdf * (np.repeat(np.repeat(E2 - E1, 4, 0), 4, 1)) / 255.0
    want_e1 = (dLdf * (1 - J / 7.0)).reshape(2, 4, 2, 4, 8).sum(axis=(1, 3))
    want_e2 = (dLdf * (J / 7.0)).reshape(2, 4, 2, 4, 8).sum(axis=(1, 3))
    np.testing.assert_allclose(gr["weights"], want_w, rtol=1e-5, atol=1e-10)
    np.testing.assert_allclose(gr["endpoints"][..., 0], want_e1, rtol=1e-5, atol=1e-10)
    np.testing.assert_allclose(gr["endpoints"][..., 1], want_e2, rtol=1e-5, atol=1e-10)


def test_adam_first_step_closed_form():
    g = np.random.default_rng(10)
    p0 = g.standard_normal(1000)
    gr = g.standard_normal(1000)
    p, m, v = O.adam_update(p0, gr, np.zeros(1000), np.zeros(1000), 1, 1e-2)
    np.testing.assert_allclose(p, p0 - 1e-2 * gr / (np.abs(gr) + 1e-8), rtol=1e-12, atol=1e-15)


def test_adam_matches_torch_optimizer():
    torch = pytest.importorskip("torch")
    g = np.random.default_rng(11)
    p0 = g.standard_normal(300)
    grads = [g.standard_normal(300) for _ in range(6)]
    tp = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(300), np.zeros(300)
    for s, gg in enumerate(grads, start=1):
        tp.grad = torch.tensor(gg, dtype=torch.float64)
        opt.step()
        p, m, v = O.adam_update(p, gg, m, v, s, 3e-3)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_train_step_projects_endpoints_and_weights():
    st = tiny_state(seed=4)
    opt = dict(step=0, lr_feat=0.5, lr_mlp=1e-3,
               m={k: np.zeros_like(st[k], dtype=np.float64) for k in ("endpoints", "weights", "grid", "mlp")},
               v={k: np.zeros_like(st[k], dtype=np.float64) for k in ("endpoints", "weights", "grid", "mlp")})
    g = np.random.default_rng(12)
    xs, ys, ks = I.train_samples(128, 8, 8, 2, g)
    tgt = g.uniform(0.0, 5.0, (128, 3))
    for _ in range(3):
        O.train_step(st, opt, xs, ys, ks, tgt)
    assert st["endpoints"].min() >= 0 and st["endpoints"].max() <= 1
    assert st["weights"].min() >= 0 and st["weights"].max() <= 1
    assert opt["step"] == 3


# ------------------------------------------------------------------------------ export

def test_export_decodes_to_bc_simulation():
    g = np.random.default_rng(13)
    W = H = 16
    ep = g.uniform(0, 1, (H // 4, W // 4, 8, 2)).astype(np.float32)
    ep[0, 0, 0] = [0.5, 0.5]           # equal endpoints
    ep[0, 1, 1] = [0.2, 0.9]           # E1 < E2 -> swapped block
    ep[1, 0, 2] = [0.9, 0.2]           # E1 > E2
    w = g.uniform(0, 1, (H, W, 8)).astype(np.float32)
    w[0, 0:4, :] = [0.0] * 8
    w[1, 0:4, :] = [1.0] * 8
    blocks = O.export_bc4(ep, w)
    dec = O.bc4_decode_blocks(blocks.reshape(-1, 8)).reshape(H // 4, W // 4, 8, 4, 4)
    y, x = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    val, *_ = O.bcsim_spatial(ep, w, x.ravel(), y.ravel())
    got = dec[y >> 2, x >> 2, :, y & 3, x & 3].reshape(-1, 8)
    np.testing.assert_array_equal(got, val)


# ------------------------------------------------------------------------------ metrics

def test_psnr_closed_form_constant_error():
    g = np.random.default_rng(14)
    tgt = g.uniform(0.0, 3.0, (2, 256, 256, 3))
    for k in range(2):
        for ty in range(2):
            for tx in range(2):
                t = tgt[k, 128 * ty:128 * ty + 128, 128 * tx:128 * tx + 128]
                t[0, 0, 0] = 0.0
                t[0, 1, 0] = 3.0 + 0.5 * tx
    delta = 0.01
    tiled, glob = O.psnr_tiled(tgt + delta, tgt)
    want = np.mean([20 * math.log10((3.0 + 0.5 * tx) / delta) for _ in range(2) for _ in range(2) for tx in range(2)])
    assert abs(tiled - want) < 1e-9
    assert abs(glob - 20 * math.log10(3.5 / delta)) < 1e-9


def test_bits_per_texel_reproduces_table3():
    rows = []
    for line in open(os.path.join(GOLDEN, "bpp_table3.txt")):
        if line.strip() and not line.startswith("#"):
            rows.append([s.strip() for s in line.split("|")])
    assert len(rows) == 4
    for name, res, hidden, printed, reproduced in rows:
        uw, uh, ut = (int(s) for s in res.split())
        bpp = O.bits_per_texel_paper(128, 128, 26, (uw, uh, ut), int(hidden))
        if reproduced == "yes":
            assert round(bpp, 2) == float(printed), (name, bpp)
        else:
            assert abs(bpp - float(printed)) < 0.05
    # the 8-channel BC4 + FP16 grid layout at the two training sizes
    assert round(O.bits_per_texel_bc4_grid(1024, 1024, 256, 256, 24), 2) == 9.33
    assert round(O.bits_per_texel_bc4_grid(4096, 4096, 1024, 1024, 48), 2) == 8.67
