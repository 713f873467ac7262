"""Pins for the CPU reference of the hybrid layout (Sec. 3.3, Eq. (4)-(5)): each test
checks it against something other than itself -- closed forms of gamma(t), printed
values of the normal CDF behind GELU, the node values of each feature map at its sample
points, exact reproduction of affine planes, the wiring of the decoder through
single-input weights, and the pinned block codec."""
import math
import os

import numpy as np

from oracle import ndgi_oracle as O
from paper_2604_12625_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _model(profile="M", keys=False, **kw):
    return I.random_hybrid_model(profile=profile, keys=keys, config=97, **kw)


def test_gamma_closed_forms():
    r3, r2 = math.sqrt(3.0) / 2, math.sqrt(2.0) / 2
    cases = {0.0: [0, 1, 0, 1], 1 / 6: [0.5, r3, r3, 0.5], 0.25: [r2, r2, 1, 0],
             0.5: [1, 0, 0, -1], 0.75: [r2, -r2, -1, 0], 1.0: [0, -1, 0, 1]}
    for t, want in cases.items():
        np.testing.assert_allclose(O.gamma_t(np.array([t]))[0], want, atol=1e-15)


def test_gelu_matches_normal_table():
    rows = [[float(s) for s in line.split("|")] for line in open(os.path.join(GOLDEN, "normal_cdf.txt"))
            if line.strip() and not line.startswith("#")]
    assert len(rows) == 9
    for x, phi in rows:
        assert abs(O.gelu(np.array([x]))[0] - x * phi) < 2e-9 * max(1.0, abs(x))
    # x Phi(x) - (-x) Phi(-x) = x because Phi(x) + Phi(-x) = 1
    x = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(O.gelu(x) - O.gelu(-x), x, atol=1e-14)


def test_key_time_coordinate():
    t = np.linspace(0.0, 1.0, 41)
    np.testing.assert_array_equal(O.key_time_coord(t, []), t)
    np.testing.assert_allclose(O.key_time_coord(t, np.arange(11) / 10.0), t, atol=1e-15)
    keys = np.array([0.0, 0.5, 0.6, 1.0])
    got = O.key_time_coord(np.array([0.25, 0.5, 0.55, 0.6, 0.8, 1.0]), keys)
    np.testing.assert_allclose(got, [1 / 6, 1 / 3, 0.5, 2 / 3, 5 / 6, 1.0], atol=1e-15)
    # before the first and after the last key the coordinate clamps
    np.testing.assert_array_equal(O.key_time_coord(np.array([0.0, 0.05, 0.95, 1.0]), [0.1, 0.9]),
                                  [0.0, 0.0, 1.0, 1.0])


def _decoded(blocks):
    """[..., 4, 8] BC4 bytes -> [..., 4 channels, 16 texels] through the pinned codec."""
    shp = blocks.shape[:-1]
    return O.bc4_decode_blocks(blocks.reshape(-1, 8)).reshape(shp + (16,))


def test_feature_maps_return_their_samples_at_sample_points():
    m = _model()
    g = np.random.default_rng(11)
    n = 400
    # F_uvt at texel centres of the Gu x Gv map and tau = k / (S - 1) (no key table)
    S, Gu, Gv = m["S"], m["Gu"], m["Gv"]
    k, y, x = g.integers(0, S, n), g.integers(0, Gv, n), g.integers(0, Gu, n)
    f = O.hybrid_features(m, (x + 0.5) / Gu, (y + 0.5) / Gv, k / (S - 1))
    dec = _decoded(m["fuvt"])                                  # [S][Gv/4][Gu/4][4][16]
    want = dec[k, y >> 2, x >> 2, :, 4 * (y & 3) + (x & 3)] / 255.0
    np.testing.assert_allclose(f[:, 0:4], want, rtol=0, atol=1e-14)
    # F_uv at texel centres of the W x H map
    W, H = m["W"], m["H"]
    y, x = g.integers(0, H, n), g.integers(0, W, n)
    f = O.hybrid_features(m, (x + 0.5) / W, (y + 0.5) / H, g.random(n))
    dec = _decoded(m["fuv"])
    np.testing.assert_allclose(f[:, 4:8], dec[y >> 2, x >> 2, :, 4 * (y & 3) + (x & 3)] / 255.0, atol=1e-14)
    # F_ut and F_vt at their texel centres and tau = k / (Tt - 1)
    U, V, Tt = m["U"], m["V"], m["Tt"]
    k, a, b = g.integers(0, Tt, n), g.integers(0, U, n), g.integers(0, V, n)
    f = O.hybrid_features(m, (a + 0.5) / U, (b + 0.5) / V, k / (Tt - 1))
    np.testing.assert_allclose(f[:, 8:10], m["fut"][k, a] / 255.0, atol=1e-14)
    np.testing.assert_allclose(f[:, 10:12], m["fvt"][k, b] / 255.0, atol=1e-14)
    np.testing.assert_allclose(f[:, 12:16], O.gamma_t(k / (Tt - 1)), atol=1e-15)


def test_planes_reproduce_affine_fields():
    m = _model()
    U, Tt = m["U"], m["Tt"]
    k, a = np.meshgrid(np.arange(Tt), np.arange(U), indexing="ij")
    m["fut"] = np.stack([10 + 2 * a + 3 * k, 200 - a - 2 * k], -1).astype(np.uint8)
    g = np.random.default_rng(12)
    u = g.uniform(1.0 / U, 1 - 1.0 / U, 500)
    t = g.random(500)
    f = O.hybrid_features(m, u, g.random(500), t)
    pa, pk = u * U - 0.5, t * (Tt - 1)
    np.testing.assert_allclose(f[:, 8] * 255, 10 + 2 * pa + 3 * pk, atol=1e-10)
    np.testing.assert_allclose(f[:, 9] * 255, 200 - pa - 2 * pk, atol=1e-10)


def test_uvt_slices_interpolate_linearly_in_time():
    m = _model()
    S, Gu, Gv = m["S"], m["Gu"], m["Gv"]
    g = np.random.default_rng(13)
    x, y = g.integers(0, Gu, 200), g.integers(0, Gv, 200)
    k = g.integers(0, S - 1, 200)
    w = g.random(200)
    u, v = (x + 0.5) / Gu, (y + 0.5) / Gv
    mid = O.hybrid_features(m, u, v, (k + w) / (S - 1))[:, 0:4]
    a = O.hybrid_features(m, u, v, k / (S - 1))[:, 0:4]
    b = O.hybrid_features(m, u, v, (k + 1) / (S - 1))[:, 0:4]
    np.testing.assert_allclose(mid, (1 - w)[:, None] * a + w[:, None] * b, atol=1e-13)


def test_key_table_warps_every_time_axis():
    m = _model(keys=True)
    keys = m["keys"].astype(np.float64)
    n = keys.size
    g = np.random.default_rng(14)
    i = g.integers(0, n - 1, 100)
    f = g.random(100)
    t = keys[i] + f * (keys[i + 1] - keys[i])
    u, v = g.random(100), g.random(100)
    plain = dict(m, keys=np.zeros(0, np.float32))
    got = O.hybrid_features(m, u, v, t)
    want = O.hybrid_features(plain, u, v, (i + f) / (n - 1))
    np.testing.assert_allclose(got[:, :12], want[:, :12], atol=1e-12)
    # gamma stays on the time itself
    np.testing.assert_allclose(got[:, 12:], O.gamma_t(t), atol=1e-15)


def test_time_clamps_and_non_finite_queries():
    m = _model(keys=True)
    q = np.array([[0.3, 0.6, -0.5], [0.3, 0.6, 0.0], [0.3, 0.6, 1.5], [0.3, 0.6, 1.0],
                  [np.nan, 0.5, 0.5], [0.5, 0.5, np.inf]], dtype=np.float32)
    out = O.hybrid_decode(m, q)
    np.testing.assert_array_equal(out[0], out[1])
    np.testing.assert_array_equal(out[2], out[3])
    assert np.isnan(out[4:]).all() and np.isfinite(out[:4]).all()


def _select_mlp(hidden, j, perm=None):
    """Decoder whose hidden unit p reads input j (layer 1), hidden-2 unit i reads hidden-1
    unit perm[i], and output c reads hidden-2 unit c."""
    P = np.zeros(O.hybrid_mlp_size(hidden))
    o1 = hidden * 16
    o3 = o1 + hidden + hidden * hidden
    o5 = o3 + hidden + 3 * hidden
    W1 = np.zeros((hidden, 16))
    W1[:, j] = np.arange(1, hidden + 1) / hidden            # unit p: x_j * (p + 1) / hidden
    W2 = np.zeros((hidden, hidden))
    perm = np.arange(hidden) if perm is None else perm
    W2[np.arange(hidden), perm] = 1.0
    W3 = np.zeros((3, hidden))
    W3[np.arange(3), np.arange(3)] = 1.0
    P[:o1] = W1.ravel()
    P[o1 + hidden:o1 + hidden + hidden * hidden] = W2.ravel()
    P[o3 + hidden:o5] = W3.ravel()
    P[o5:] = [0.5, -0.25, 0.0]
    return P


def test_decoder_wiring_and_orientation():
    for hidden in (16, 64):
        m = _model("M.64" if hidden == 64 else "M")
        perm = np.roll(np.arange(hidden), -5)
        m["mlp"] = _select_mlp(hidden, 13, perm)                  # input 13 = cos(pi t)
        t = np.array([0.0, 1 / 3, 0.5, 0.9])
        out = O.hybrid_decode_f64(m, np.full(4, 0.3), np.full(4, 0.7), t)
        c = np.cos(np.pi * t)
        for r in range(3):
            scale = (perm[r] + 1) / hidden
            np.testing.assert_allclose(out[:, r], O.gelu(O.gelu(c * scale)) + [0.5, -0.25, 0.0][r],
                                       atol=1e-15)


def test_hybrid_page_decode_equals_texel_centre_queries():
    m = _model(keys=True)
    t = np.float32(0.41)
    dst = np.zeros((128 * 128, 3))
    bad = O.hybrid_decode_pages([m], [(0, 0, 0, t, 0), (0, 1, 0, t, 0), (2, 0, 0, t, 0)], 128, dst, 128)
    assert bad == 2
    y, x = np.meshgrid(np.arange(128), np.arange(128), indexing="ij")
    q = np.stack([((x + 0.5) / 128).ravel(), ((y + 0.5) / 128).ravel(), np.full(128 * 128, t)], 1)
    np.testing.assert_allclose(dst, O.hybrid_decode(m, q.astype(np.float32)), rtol=1e-13, atol=1e-15)


def test_mirror_texel_is_numpys_symmetric_padding():
    """Mirror addressing equals numpy's 'symmetric' padding of an index ramp (the edge
    texel repeated, then the map reflected)."""
    for n, b in ((8, 4), (128, 4), (37, 32), (5, 5)):
        np.testing.assert_array_equal(O.mirror_texel(np.arange(-b, n + b), n),
                                      np.pad(np.arange(n), b, mode="symmetric"))


def test_bordered_pages_mirror_tiles_and_join_neighbours():
    """A per-tile model's bordered page is its plain page padded symmetrically (the border
    mirrors the tile, supplementary Virtual Texturing section); on a map of several pages the border of an inner page holds
    the neighbouring pages' texels, so the pages join without seams; the interior is the
    plain page."""
    b, t = 4, np.float32(0.63)
    m = _model(keys=True)                                    # one 128^2 tile model
    plain = np.zeros((128 * 128, 3))
    O.hybrid_decode_pages([m], [(0, 0, 0, t, 0)], 128, plain, 128)
    R = 128 + 2 * b
    bord = np.zeros((R * R, 3))
    assert O.hybrid_decode_pages([m], [(0, 0, 0, t, 0)], 128, bord, R, border=b) == 0
    np.testing.assert_array_equal(bord.reshape(R, R, 3),
                                  np.pad(plain.reshape(128, 128, 3), ((b, b), (b, b), (0, 0)), mode="symmetric"))
    big = I.random_hybrid_model(256, 256, profile="L", plane=(64, 64, 6), config=31, uvt_side=(32, 32))
    pages = np.zeros((256 * 256, 3))                          # the whole map as 2 x 2 plain pages
    O.hybrid_decode_pages([big], [(0, px, py, t, py * 128 * 256 + px * 128) for py in (0, 1) for px in (0, 1)], 128,
                          pages, 256)
    full = pages.reshape(256, 256, 3)
    bord = np.zeros((R * R, 3))
    O.hybrid_decode_pages([big], [(0, 1, 0, t, 0)], 128, bord, R, border=b)
    bord = bord.reshape(R, R, 3)
    padded = np.pad(full, ((b, b), (b, b), (0, 0)), mode="symmetric")
    np.testing.assert_array_equal(bord, padded[0:R, 128:128 + R])
    np.testing.assert_array_equal(bord[b:b + 128, b:b + 128], full[0:128, 128:256])


# ----------------------------------------------------------------- hybrid training pins
def tiny_hybrid_state(hidden=16, seed=0, frames=3, keys=True, on_grid=False):
    """A small trainable hybrid state: 8 x 8 map, F_uvt 4 x 4 x 3, planes 4 x 3."""
    g = np.random.default_rng(seed)
    W = H = 8
    Gu = Gv = 4
    S, U, V, Tt = 3, 4, 4, 3
    kt = np.sort(g.uniform(0, 1, frames)).astype(np.float32) if keys else np.zeros(0, np.float32)
    st = dict(dims=dict(W=W, H=H, Gu=Gu, Gv=Gv, S=S, U=U, V=V, Tt=Tt, hidden=hidden, frames=frames, keys=kt))
    st["fuv_ep"] = g.uniform(0, 1, (H // 4, W // 4, 4, 2))
    st["fuv_w"] = g.uniform(0, 1, (H, W, 4))
    st["fuvt_ep"] = g.uniform(0, 1, (S, Gv // 4, Gu // 4, 4, 2))
    st["fuvt_w"] = g.uniform(0, 1, (S, Gv, Gu, 4))
    if on_grid:
        # endpoints on the 8-bit grid and weights 0 or 1: the simulated value equals the lerp
        for k in ("fuv_ep", "fuvt_ep"):
            st[k] = g.integers(0, 256, st[k].shape) / 255.0
        for k in ("fuv_w", "fuvt_w"):
            st[k] = g.integers(0, 2, st[k].shape).astype(np.float64)
    st["fut"] = g.uniform(0, 1, (Tt, U, 2))
    st["fvt"] = g.uniform(0, 1, (Tt, V, 2))
    st["mlp"] = I.hybrid_mlp(hidden, np.float64, g)
    for k in O.HYB_KEYS:
        st[k] = np.asarray(st[k], dtype=np.float64)
    return st


def _batch(st, n, seed):
    g = np.random.default_rng(seed)
    d = st["dims"]
    return g.integers(0, d["W"], n), g.integers(0, d["H"], n), g.integers(0, d["frames"], n), g.normal(0, 1, (n, 3))


def test_splitmix64_published_outputs_and_noise_range():
    # the generator's first two outputs from state 0 (reference implementation of SplitMix64)
    assert int(O.splitmix64(0)) == 0xE220A8397B1DCDAF
    assert int(O.splitmix64(0x9E3779B97F4A7C15)) == 0x6E789E6AA1B965F4
    z = O.hybrid_noise(7, 3, np.arange(20000)[:, None], np.arange(12)[None, :])
    assert z.min() >= -0.5 and z.max() < 0.5
    assert abs(z.mean()) < 5e-3 and abs(z.var() - 1 / 12) < 2e-3
    assert not np.array_equal(z, O.hybrid_noise(7, 4, np.arange(20000)[:, None], np.arange(12)[None, :]))


def _fd_check(st, xs, ys, fs, tgt, flags, keys, h=1e-6, n_probe=12, seed=5):
    loss, g = O.hybrid_train_grads(st, xs, ys, fs, tgt, flags, seed=9, step=2)
    rng = np.random.default_rng(seed)
    for key in keys:
        a = st[key]
        flat = a.reshape(-1)
        gflat = g[key].reshape(-1)
        idx = np.argsort(-np.abs(gflat))[:n_probe // 2]
        idx = np.concatenate([idx, rng.integers(0, flat.size, n_probe - idx.size)])
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = O.hybrid_train_grads(st, xs, ys, fs, tgt, flags, seed=9, step=2)[0]
            flat[i] = old - h
            lm = O.hybrid_train_grads(st, xs, ys, fs, tgt, flags, seed=9, step=2)[0]
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (key, int(i), fd, gflat[i])


def test_hybrid_gradients_match_finite_differences():
    for hidden in (16, 64):
        st = tiny_hybrid_state(hidden, seed=hidden)
        xs, ys, fs, tgt = _batch(st, 40, seed=hidden + 1)
        # continuous features (no simulation): every array; with noise on, fixed draws
        _fd_check(st, xs, ys, fs, tgt, O.HT_NOISE, O.HYB_KEYS)
        # under the simulation the decoder and the planes still have exact derivatives
        _fd_check(st, xs, ys, fs, tgt, O.HT_BCSIM | O.HT_NOISE, ("mlp", "fut", "fvt"))


def test_straight_through_gradient_is_the_lerp_gradient_on_the_grid():
    st = tiny_hybrid_state(16, seed=3, on_grid=True)
    xs, ys, fs, tgt = _batch(st, 50, seed=4)
    l1, g1 = O.hybrid_train_grads(st, xs, ys, fs, tgt, O.HT_BCSIM)
    l0, g0 = O.hybrid_train_grads(st, xs, ys, fs, tgt, 0)
    assert abs(l1 - l0) < 1e-12
    for k in O.HYB_KEYS:
        np.testing.assert_allclose(g1[k], g0[k], atol=1e-12)


def test_export_decodes_to_the_simulated_forward():
    st = tiny_hybrid_state(64, seed=6)
    for k in ("fut", "fvt"):
        st[k] = np.asarray(st[k], dtype=np.float32).astype(np.float64)
    m = O.hybrid_export(st)
    d = st["dims"]
    y, x = np.meshgrid(np.arange(d["H"]), np.arange(d["W"]), indexing="ij")
    for f in range(d["frames"]):
        n = x.size
        fwd = O.hybrid_train_forward(st, x.ravel(), y.ravel(), np.full(n, f), O.HT_BCSIM | O.HT_QPLANES)
        t = np.full(n, np.float64(d["keys"][f]))
        dec = O.hybrid_decode_f64(m, (x.ravel() + 0.5) / d["W"], (y.ravel() + 0.5) / d["H"], t)
        np.testing.assert_allclose(dec, fwd, rtol=0, atol=1e-12)


def test_target_normalisation_closed_form():
    tgt = np.stack([np.full((4, 4, 3), 2.0), np.full((4, 4, 3), 0.5)])
    tgt[1, :, :, 2] = 8.0
    y, means = O.hybrid_normalise_target(tgt, 2.2)
    np.testing.assert_allclose(y, 1.0, atol=1e-15)
    np.testing.assert_allclose(means[0], 2.0 ** (1 / 2.2), rtol=1e-15)
    np.testing.assert_allclose(means[1], [0.5 ** (1 / 2.2), 0.5 ** (1 / 2.2), 8.0 ** (1 / 2.2)], rtol=1e-15)
    np.testing.assert_allclose(O.hybrid_restore(y[1, 0, 0], means[1], 2.2), [0.5, 0.5, 8.0], rtol=1e-14)


# ------------------------------------------------------------------------ BC7 mode 6
def _golden_bc7():
    rows = []
    for line in open(os.path.join(GOLDEN, "bc7_mode6_blocks.txt")):
        if line.strip() and not line.startswith("#"):
            a, b = line.split("|")
            vals = np.array([int(x) for x in b.split()], dtype=np.uint8).reshape(4, 16).T   # [texel][channel]
            rows.append((np.array([int(h, 16) for h in a.split()], dtype=np.uint8), vals))
    return rows


def test_bc7_golden_blocks():
    rows = _golden_bc7()
    assert len(rows) == 3
    ys, xs = np.meshgrid(np.arange(4), np.arange(4), indexing="ij")
    for blk, want in rows:
        np.testing.assert_array_equal(O.bc7m6_decode_block(blk), want)
        got = O.bc7_texels(np.repeat(blk[None], 16, 0), xs.ravel(), ys.ravel())
        np.testing.assert_array_equal(got, want)


def test_bc7_equal_endpoints_and_symmetric_weights():
    g = np.random.default_rng(30)
    for _ in range(200):
        blk = I.random_bc7m6((), g)
        E0, E1, idx = O.bc7m6_fields(blk)
        dec = O.bc7m6_decode_block(blk)
        # weights are symmetric: swapping the endpoints and replacing index j by 15 - j leaves
        # every texel unchanged (the reading the export's anchor rule relies on)
        for s_ in range(16):
            w, w2 = O.BC7_WEIGHTS4[idx[s_]], O.BC7_WEIGHTS4[15 - idx[s_]]
            assert w + w2 == 64
            for c in range(4):
                assert dec[s_, c] == ((64 - w2) * E1[c] + w2 * E0[c] + 32) >> 6
                lo, hi = min(E0[c], E1[c]), max(E0[c], E1[c])
                assert lo <= dec[s_, c] <= hi


def test_bc7_export_decodes_to_the_simulation():
    g = np.random.default_rng(31)
    ep = g.uniform(0, 1, (3, 5, 4, 2))
    w = g.uniform(0, 1, (12, 20))
    w[0, 0] = 0.99          # anchor index >= 8 in block (0, 0): the export swaps
    w[4, 4] = 0.01
    blocks = O.export_bc7(ep, w)
    E1 = O.bc7_quantise_endpoint(ep[..., 0])[0]
    E2 = O.bc7_quantise_endpoint(ep[..., 1])[0]
    J = O.quantise_weight4(w)
    for by in range(3):
        for bx in range(5):
            dec = O.bc7m6_decode_block(blocks[by, bx])
            for s_ in range(16):
                y, x = 4 * by + s_ // 4, 4 * bx + s_ % 4
                wj = O.BC7_WEIGHTS4[J[y, x]]
                want = ((64 - wj) * E1[by, bx] + wj * E2[by, bx] + 32) >> 6
                np.testing.assert_array_equal(dec[s_], want)
    assert O.bc7m6_fields(blocks[0, 0])[2][0] < 8


def test_bc7_pbit_quantisation():
    # all four channels sit on odd 8-bit values: p = 1 reproduces them exactly
    e = np.array([[13, 201, 77, 255]]) / 255.0
    E, v7, p = O.bc7_quantise_endpoint(e)
    assert p[0] == 1 and list(E[0]) == [13, 201, 77, 255]
    e = np.array([[12, 200, 76, 254]]) / 255.0
    E, v7, p = O.bc7_quantise_endpoint(e)
    assert p[0] == 0 and list(E[0]) == [12, 200, 76, 254]
    # mixed parities: every channel within 1 of its target
    g = np.random.default_rng(32)
    e = g.uniform(0, 1, (1000, 4))
    E, v7, p = O.bc7_quantise_endpoint(e)
    assert np.all(np.abs(E - np.float32(255) * e.astype(np.float32)) <= 1.0 + 1e-6)
    assert np.all(E == 2 * v7 + p[:, None])


def test_bc7_hybrid_gradients_and_export():
    st = tiny_hybrid_state(16, seed=33)
    st["dims"] = dict(st["dims"], codec=1)
    g = np.random.default_rng(34)
    st["fuv_w"] = g.uniform(0, 1, st["fuv_w"].shape[:2])
    st["fuvt_w"] = g.uniform(0, 1, st["fuvt_w"].shape[:3])
    xs, ys, fs, tgt = _batch(st, 40, seed=35)
    _fd_check(st, xs, ys, fs, tgt, O.HT_NOISE, O.HYB_KEYS)
    _fd_check(st, xs, ys, fs, tgt, O.HT_BCSIM | O.HT_NOISE, ("mlp", "fut", "fvt"))
    for k in ("fut", "fvt"):
        st[k] = np.asarray(st[k], dtype=np.float32).astype(np.float64)
    m = O.hybrid_export(st)
    assert m["fuv"].shape == (2, 2, 16) and m["codec"] == 1
    d = st["dims"]
    y, x = np.meshgrid(np.arange(d["H"]), np.arange(d["W"]), indexing="ij")
    for f in range(d["frames"]):
        n = x.size
        fwd = O.hybrid_train_forward(st, x.ravel(), y.ravel(), np.full(n, f), O.HT_BCSIM | O.HT_QPLANES)
        dec = O.hybrid_decode_f64(m, (x.ravel() + 0.5) / d["W"], (y.ravel() + 0.5) / d["H"],
                                  np.full(n, np.float64(d["keys"][f])))
        np.testing.assert_allclose(dec, fwd, rtol=0, atol=1e-12)
