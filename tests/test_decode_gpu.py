"""GPU parity of the decode path against the CPU oracle, through the C ABI.

Tolerances: BC4 decode bit-exact; decoded RGB within 1e-5 (FP32 path) and 2e-3 (FP16
MFMA path) relative per channel, max over the compared set."""
import numpy as np
import pytest

from oracle import ndgi_oracle as O
from paper_2604_12625_amd import inputs as I
from tests.gpu_util import assert_rel, torch_cuda

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL16 = 2e-3


@pytest.fixture(scope="module")
def N():
    torch_cuda()
    from paper_2604_12625_amd import ndgi
    return ndgi


@pytest.fixture(scope="module")
def ctx(N):
    c = N.Context(0)
    yield c
    c.close()


def _dec(N, ctx, model, q, prec):
    import torch
    dm = N.DeviceModel.from_numpy(model)
    out = ctx.decode(dm, torch.from_numpy(q).cuda(), prec)
    torch.cuda.synchronize()
    return out.float().cpu().numpy()


# ------------------------------------------------------------------------------ BC4
def test_bc4_blocks_bit_exact(N):
    import torch
    from tests.test_oracle import _golden_blocks
    gold = _golden_blocks()
    blocks = np.stack([b for b, _ in gold])
    out = N.bc4_decode_blocks(torch.from_numpy(blocks).cuda()).cpu().numpy()
    np.testing.assert_array_equal(out, np.stack([w for _, w in gold]))
    g = np.random.default_rng(20)
    rnd = g.integers(0, 256, size=(1_000_003, 8), dtype=np.uint8)
    out = N.bc4_decode_blocks(torch.from_numpy(rnd).cuda()).cpu().numpy()
    np.testing.assert_array_equal(out, O.bc4_decode_blocks(rnd))
    empty = torch.empty((0, 8), dtype=torch.uint8, device="cuda")
    assert N.bc4_decode_blocks(empty).shape == (0, 16)


@pytest.mark.parametrize("impl", [0, 1, 2])
def test_kernel_bc4_decoders_exhaustive(N, impl):
    """Every (e0, e1) pair with every selector at every texel position (8 blocks per pair,
    selector (s + k) mod 8 at texel s), through each texel decoder the kernels use, equals
    the oracle's palette byte for byte."""
    import torch
    e = np.arange(65536)
    blocks = np.zeros((65536, 8, 8), dtype=np.uint8)
    for k in range(8):
        field = 0
        for s_ in range(16):
            field |= ((s_ + k) % 8) << (3 * s_)
        blocks[:, k, 0] = e >> 8
        blocks[:, k, 1] = e & 255
        blocks[:, k, 2:] = np.frombuffer(field.to_bytes(6, "little"), np.uint8)
    blocks = blocks.reshape(-1, 8)
    out = N.bc4_decode_blocks(torch.from_numpy(blocks).cuda(), impl=impl).cpu().numpy()
    np.testing.assert_array_equal(out, O.bc4_decode_blocks(blocks))


# --------------------------------------------------------------------------- decode
def c1_model():
    """64x64 map, grid 16x16x8(t)x8 FP32 U[-1,1], He-normal FP32 decoder (seed 0)."""
    return I.random_model(64, 64, 16, 16, 8, np.float32, np.float32, config=1)


def test_decode_c1_fp32_all_texel_centres(N, ctx):
    m = c1_model()
    ts = I.rng(1, I.P_QUERY).random(8, dtype=np.float32)
    q = I.texel_centre_queries(64, 64, ts)
    assert q.shape == (32768, 3)
    assert_rel(_dec(N, ctx, m, q, N.PREC_F32), O.decode(m, q), TOL32, "C1 FP32")


@pytest.mark.parametrize("prec,tol", [(1, TOL16), (0, TOL32)])
def test_decode_fp16_model_centres_and_random(N, ctx, prec, tol):
    m = I.random_model(256, 192, 64, 48, 24, np.float16, np.float16, config=50)
    q1 = I.texel_centre_queries(256, 192, [0.0, 0.61])
    q2 = I.uniform_queries(70001, I.rng(50, I.P_QUERY))
    q = np.concatenate([q1, q2])
    assert_rel(_dec(N, ctx, m, q, prec), O.decode(m, q), tol, f"prec {prec}")


@pytest.mark.parametrize("n", [1, 15, 63, 64, 65, 1000])
@pytest.mark.parametrize("prec", [0, 1])
def test_decode_ragged_counts(N, ctx, n, prec):
    m = I.random_model(64, 64, 16, 16, 8, np.float16, np.float16, config=51)
    q = I.uniform_queries(n, I.rng(51, I.P_QUERY, n))
    assert_rel(_dec(N, ctx, m, q, prec), O.decode(m, q), TOL16 if prec else TOL32, f"n={n}")


def test_decode_edges_clamp_wrap_nan(N, ctx):
    m = I.random_model(128, 64, 32, 16, 12, np.float16, np.float16, config=52)
    q = np.array([[-0.5, 0.5, 0.2], [1.7, 0.5, 0.2], [0.5, -3.0, 0.2], [0.5, 9.0, 0.2],
                  [0.0, 0.0, 0.0], [0.999999, 0.999999, 0.999999], [0.3, 0.4, -0.25],
                  [0.3, 0.4, 7.75], [0.3, 0.4, 11.0 / 12.0 + 1e-4], [0.25, 0.75, 0.999]],
                 dtype=np.float32)
    bad = np.array([[np.nan, 0.5, 0.2], [0.5, np.inf, 0.2], [0.5, 0.5, -np.inf]], dtype=np.float32)
    for prec, tol in ((0, TOL32), (1, TOL16)):
        assert_rel(_dec(N, ctx, m, q, prec), O.decode(m, q), tol, "edges")
        assert np.isnan(_dec(N, ctx, m, bad, prec)).all()


def test_decode_argument_errors(N, ctx):
    import ctypes
    import torch
    m = I.random_model(64, 64, 16, 16, 8, np.float16, np.float16, config=53)
    dm = N.DeviceModel.from_numpy(m)
    q = torch.zeros((4, 3), device="cuda")
    with pytest.raises(N.NdgiError):
        ctx.decode(dm, q, prec=7)
    dm.desc.W = 62
    with pytest.raises(N.NdgiError, match="multiples of 4"):
        ctx.decode(dm, q, N.PREC_F32)
    dm.desc.W = 64
    rc = N.lib().ndgi_decode(ctx.h, ctypes.byref(dm.desc), None, 4, None, 0, None)
    assert rc == N.ERR_INVALID_ARG


# --------------------------------------------------------------------------- binned
def _dec_binned(N, ctx, model, q, prec, ws=None):
    import torch
    dm = N.DeviceModel.from_numpy(model)
    out, ws = ctx.decode_binned(dm, torch.from_numpy(q).cuda(), prec, workspace=ws)
    torch.cuda.synchronize()
    return out.float().cpu().numpy(), ws


EDGE_Q = np.array([[-0.5, 0.5, 0.2], [1.7, 0.5, 0.2], [0.5, -3.0, 0.2], [0.5, 9.0, 0.2],
                   [0.0, 0.0, 0.0], [0.999999, 0.999999, 0.999999], [0.3, 0.4, -0.25],
                   [1.0, 1.0, 0.5], [0.3, 0.4, 7.75], [0.25, 0.75, 0.999]], dtype=np.float32)
BAD_Q = np.array([[np.nan, 0.5, 0.2], [0.5, np.inf, 0.2], [0.5, 0.5, -np.inf],
                  [-np.inf, np.nan, 0.1], [np.inf, np.inf, 0.3]], dtype=np.float32)


@pytest.mark.parametrize("prec,tol", [(1, TOL16), (0, TOL32)])
@pytest.mark.parametrize("grid_dt", [np.float16, np.float32])
@pytest.mark.parametrize("grid", [(50, 37), (70, 30)])
def test_binned_equals_direct_and_oracle(N, ctx, prec, tol, grid_dt, grid):
    """Several tiles with a ragged edge (200 x 148 texels), all texel centres at one time,
    random queries, out-of-range and non-finite queries: the binned decode gives the direct
    decode's bits and the oracle's values.  A 50 x 37 grid (a quarter of the texel
    resolution) bins by 8 x 8 grid cells, a 70 x 30 grid by 32 x 32 texel tiles."""
    m = I.random_model(200, 148, grid[0], grid[1], 12, grid_dt, np.float16, config=54)
    q = np.concatenate([I.texel_centre_queries(200, 148, [0.37]),
                        I.uniform_queries(50001, I.rng(54, I.P_QUERY)), EDGE_Q, BAD_Q])
    direct = _dec(N, ctx, m, q, prec)
    binned, _ = _dec_binned(N, ctx, m, q, prec)
    np.testing.assert_array_equal(binned, direct)
    ok = np.isfinite(q).all(axis=1)
    assert np.isnan(binned[~ok]).all()
    assert_rel(binned[ok], O.decode(m, q[ok]), tol, f"binned prec {prec}")


@pytest.mark.parametrize("grid_dt", [np.float16, np.float32])
def test_binned_long_time_axis(N, ctx, grid_dt):
    """T = 64 keys: the tile's grid window over all keys exceeds the LDS budget, so the
    decode reads nodes from HBM in time-key order; still the direct decode's bits."""
    m = I.random_model(128, 96, 32, 24, 64, grid_dt, np.float16, config=57)
    q = np.concatenate([I.uniform_queries(40000, I.rng(57, I.P_QUERY)), EDGE_Q])
    for prec, tol in ((1, TOL16), (0, TOL32)):
        direct = _dec(N, ctx, m, q, prec)
        binned, _ = _dec_binned(N, ctx, m, q, prec)
        np.testing.assert_array_equal(binned, direct)
        sel = np.random.default_rng(57).integers(0, q.shape[0], 4096)
        assert_rel(binned[sel], O.decode(m, q[sel]), tol, f"T=64 prec {prec}")


@pytest.mark.parametrize("T", [24, 25, 31])
def test_binned_lds_window_capacities(N, ctx, T):
    """Grid-aligned tiles (9 x 9 nodes per key) with windows up to the largest that the
    LDS-staged decode takes (T = 31: 2511 of its 2560 uint4); queries reach the region's
    first and last texel rows and columns (map edges, non-finite inputs)."""
    m = I.random_model(256, 160, 64, 40, T, np.float16, np.float16, config=60)
    q = np.concatenate([I.uniform_queries(30000, I.rng(60, I.P_QUERY, T)), EDGE_Q, BAD_Q,
                        I.texel_centre_queries(256, 160, [0.61])])
    for prec, tol in ((1, TOL16), (0, TOL32)):
        direct = _dec(N, ctx, m, q, prec)
        binned, _ = _dec_binned(N, ctx, m, q, prec)
        np.testing.assert_array_equal(binned, direct)
        ok = np.isfinite(q).all(axis=1)
        sel = np.flatnonzero(ok)[np.random.default_rng(60).integers(0, ok.sum(), 2048)]
        assert_rel(binned[sel], O.decode(m, q[sel]), tol, f"T={T} prec {prec}")


@pytest.mark.parametrize("T", [2, 3])
def test_binned_full_resolution_grid_window(N, ctx, T):
    """A grid at the texel resolution: a 32-texel tile's window is 35 x 35 nodes, more nodes
    per key than a workgroup stages per round, so the staging walk advances by less than one
    key per round (T = 2 fits the LDS window; T = 3 does not and reads nodes from HBM)."""
    m = I.random_model(160, 100, 160, 100, T, np.float16, np.float16, config=58)
    q = np.concatenate([I.uniform_queries(30000, I.rng(58, I.P_QUERY, T)), EDGE_Q])
    for prec, tol in ((1, TOL16), (0, TOL32)):
        direct = _dec(N, ctx, m, q, prec)
        binned, _ = _dec_binned(N, ctx, m, q, prec)
        np.testing.assert_array_equal(binned, direct)
        sel = np.random.default_rng(58).integers(0, q.shape[0], 2048)
        assert_rel(binned[sel], O.decode(m, q[sel]), tol, f"full-resolution grid T={T} prec {prec}")


@pytest.mark.parametrize("n", [1, 2, 63, 65, 1023, 1025, 4097])
def test_binned_ragged_counts_reuse_workspace(N, ctx, n):
    """Counts around the wave (64) and chunk (1024) sizes; one workspace serves calls of
    decreasing size in a row, and its stale contents do not leak into later results."""
    m = I.random_model(96, 64, 24, 16, 8, np.float16, np.float16, config=55)
    q_big = I.uniform_queries(9000, I.rng(55, I.P_QUERY, 0))
    _, ws = _dec_binned(N, ctx, m, q_big, 1)
    q = I.uniform_queries(n, I.rng(55, I.P_QUERY, n))
    got, ws2 = _dec_binned(N, ctx, m, q, 1, ws)
    assert ws2 is ws
    np.testing.assert_array_equal(got, _dec(N, ctx, m, q, 1))
    assert_rel(got, O.decode(m, q), TOL16, f"n={n}")


def test_binned_item_map_beyond_staging(N, ctx):
    """36M queries over 6 tiles: 17,580 work items, more than the bin scan stages in LDS
    (17,408), so the item -> bin map is written straight from the scan's runs."""
    m = I.random_model(96, 64, 24, 16, 8, np.float16, np.float16, config=59)
    q = I.uniform_queries(36_000_000, I.rng(59, I.P_QUERY))
    got, _ = _dec_binned(N, ctx, m, q, 1)
    direct = _dec(N, ctx, m, q, 1)
    assert np.array_equal(got, direct)
    del direct
    sel = np.random.default_rng(59).integers(0, q.shape[0], 4096)
    assert_rel(got[sel], O.decode(m, q[sel]), TOL16, "item map beyond staging")


def test_binned_64_texel_tiles(N, ctx):
    """A map of more than 16384 tiles of 32^2 texels (8192 x 2112) bins by 64^2 tiles."""
    import torch
    m = I.random_model(8192, 2112, 2048, 528, 4, np.float16, np.float16, config=56)
    assert ctx.binned_workspace_bytes(N.DeviceModel.from_numpy(m), 0) == 512 * 128 * 33 * 4 + \
        2 * (((128 * 33 + 1) * 4 + 255) // 256 * 256) + (4 * 128 * 33 + 255) // 256 * 256 + 4096
    q = I.uniform_queries(300_000, I.rng(56, I.P_QUERY))
    got, _ = _dec_binned(N, ctx, m, q, 1)
    np.testing.assert_array_equal(got, _dec(N, ctx, m, q, 1))
    sel = np.random.default_rng(56).integers(0, q.shape[0], 4096)
    assert_rel(got[sel], O.decode(m, q[sel]), TOL16, "64^2 tiles")
    del torch


def test_reserved_decode_takes_the_binned_route(N):
    """ndgi_decode on a context with a reserved workspace: at 100+ queries per tile it runs
    the binned kernels, below that or when the reservation is too small the query-order pass;
    every route gives the unreserved decode's bits, and the oracle's values on a sample."""
    import torch
    m = I.random_model(1024, 1024, 256, 256, 24, np.float16, np.float16, config=73)   # 1024 tiles
    dm = N.DeviceModel.from_numpy(m)
    plain = N.Context(0)
    res = N.Context(0)
    try:
        q_big = torch.from_numpy(I.uniform_queries(300_000, I.rng(73, I.P_QUERY, 0))).cuda()   # 293 per tile
        q_small = torch.from_numpy(I.uniform_queries(50_000, I.rng(73, I.P_QUERY, 1))).cuda()  # below 100 per tile
        res.reserve_decode(dm, 300_000)
        for prec, tol in ((1, TOL16), (0, TOL32)):
            for q in (q_big, q_small):
                want = plain.decode(dm, q, prec)
                got = res.decode(dm, q, prec)
                torch.cuda.synchronize()
                assert torch.equal(got.view(torch.int16 if prec else torch.int32),
                                   want.view(torch.int16 if prec else torch.int32)), (prec, q.shape[0])
            sel = np.random.default_rng(73).integers(0, q_big.shape[0], 2048)
            g = res.decode(dm, q_big, prec).float().cpu().numpy()
            assert_rel(g[sel], O.decode(m, q_big.cpu().numpy()[sel]), tol, f"reserved prec {prec}")
        # a reservation too small for the batch: the query-order pass, same bits
        res.reserve_decode(None, 0)
        res.reserve_decode(dm, 120_000)
        got = res.decode(dm, q_big, 1)
        want = plain.decode(dm, q_big, 1)
        torch.cuda.synchronize()
        assert torch.equal(got.view(torch.int16), want.view(torch.int16))
        with pytest.raises(N.NdgiError):
            res.reserve_decode(dm, -1)
    finally:
        plain.close()
        res.close()


def test_binned_argument_errors(N, ctx):
    import ctypes
    import torch
    m = I.random_model(64, 64, 16, 16, 8, np.float16, np.float16, config=53)
    dm = N.DeviceModel.from_numpy(m)
    q = torch.rand((100, 3), device="cuda")
    out = torch.empty((100, 3), dtype=torch.float16, device="cuda")
    need = ctx.binned_workspace_bytes(dm, 100)
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    L = N.lib()
    args = (ctx.h, ctypes.byref(dm.desc), q.data_ptr(), 100, out.data_ptr(), 1)
    assert L.ndgi_decode_binned(*args, ws.data_ptr(), need - 1, None) == N.ERR_INVALID_ARG
    assert b"needed" in L.ndgi_last_error()
    assert L.ndgi_decode_binned(*args, ws.data_ptr() + 16, need, None) == N.ERR_INVALID_ARG
    assert L.ndgi_decode_binned(*args, None, need, None) == N.ERR_INVALID_ARG
    assert L.ndgi_decode_binned(ctx.h, ctypes.byref(dm.desc), q.data_ptr(), 100, out.data_ptr(), 5,
                                ws.data_ptr(), need, None) == N.ERR_INVALID_ARG
    assert L.ndgi_decode_binned(ctx.h, ctypes.byref(dm.desc), None, 0, None, 1, None, 0, None) == N.OK
    assert L.ndgi_decode_binned(*args, ws.data_ptr(), need, None) == N.OK
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------- pages
def _vt_setup(prec, seed=60):
    sides = [(256, 256, 24), (384, 384, 24), (512, 256, 12)]
    models = [I.random_model(W, H, W // 4, H // 4, T, np.float16, np.float16, config=seed, index=i)
              for i, (W, H, T) in enumerate(sides)]
    g = I.rng(seed, I.P_REQ)
    reqs = []
    for r in range(24):
        mi = int(g.integers(0, 3))
        W, H, _ = sides[mi]
        reqs.append((mi, int(g.integers(0, W // 128)), int(g.integers(0, H // 128)),
                     float(g.random(dtype=np.float32)), 0))
    reqs += [(3, 0, 0, 0.5, 0), (-1, 0, 0, 0.5, 0), (0, 2, 0, 0.5, 0), (2, 3, 2, 0.5, 0), (1, -1, 0, 0.1, 0)]
    # physical texture: 8 pages per row
    reqs = [(m, px, py, t, (i // 8) * 128 * 1024 + (i % 8) * 128) for i, (m, px, py, t, _) in enumerate(reqs)]
    return models, reqs


def _run_pages(N, ctx, models, reqs, prec, graph=False, n_serve=None, dst=None):
    import torch
    dms = [N.DeviceModel.from_numpy(m) for m in models]
    marr = N.models_array(dms)
    r = np.array(reqs, dtype=object)
    rq = N.page_requests(r[:, 0].astype(np.int32), r[:, 1].astype(np.int32), r[:, 2].astype(np.int32),
                         r[:, 3].astype(np.float32), r[:, 4].astype(np.int64))
    nreq = torch.tensor([len(reqs) if n_serve is None else n_serve], dtype=torch.int32, device="cuda")
    rows = ((len(reqs) + 7) // 8) * 128
    dt = torch.float16 if prec == 1 else torch.float32
    if dst is None:
        dst = torch.full((rows * 1024, 3), -7.0, dtype=dt, device="cuda")
    ctx.decode_pages(marr, len(models), rq, nreq, len(reqs), 128, dst, 1024, prec, graph=graph)
    torch.cuda.synchronize()
    return dst.float().cpu().numpy(), (dms, marr, rq, nreq)


@pytest.mark.parametrize("prec,tol", [(1, TOL16), (0, TOL32)])
def test_pages_many_models_and_bad_requests(N, ctx, prec, tol):
    models, reqs = _vt_setup(prec)
    out, _ = _run_pages(N, ctx, models, reqs, prec)
    assert ctx.error_flags() & N.FLAG_BAD_PAGE_REQUEST
    assert ctx.error_flags() == 0                      # reading clears the flags
    rows = out.shape[0] // 1024
    ref = np.full((rows * 1024, 3), -7.0)
    bad = O.decode_pages(models, reqs, 128, ref, 1024)
    assert bad == 5
    valid = ref[:, 0] != -7.0
    assert_rel(out[valid], ref[valid], tol, "pages")
    np.testing.assert_array_equal(out[~valid], -7.0)


def test_pages_graph_replay_with_new_requests(N, ctx):
    import torch
    models, reqs = _vt_setup(1, seed=61)
    reqs = reqs[:24]
    out1, keep = _run_pages(N, ctx, models, reqs, 1, graph=True)
    dms, marr, rq, nreq = keep
    ref = np.full(out1.shape, -7.0)
    O.decode_pages(models, reqs, 128, ref, 1024)
    assert_rel(out1[ref[:, 0] != -7.0], ref[ref[:, 0] != -7.0], TOL16, "graph #1")
    # new times and a smaller count in the same device buffers, replay
    reqs2 = [(m, px, py, (t + 0.37) % 1.0, off) for (m, px, py, t, off) in reqs]
    r = np.array(reqs2, dtype=object)
    rq.copy_(N.page_requests(r[:, 0].astype(np.int32), r[:, 1].astype(np.int32), r[:, 2].astype(np.int32),
                             r[:, 3].astype(np.float32), r[:, 4].astype(np.int64)))
    nreq.fill_(16)
    dst = torch.full((out1.shape[0], 3), -7.0, dtype=torch.float16, device="cuda")
    for _ in range(3):
        ctx.decode_pages(marr, len(models), rq, nreq, len(reqs), 128, dst, 1024, 1, graph=True)
        torch.cuda.synchronize()
        out2 = dst.float().cpu().numpy()
        ref2 = np.full(out1.shape, -7.0)
        O.decode_pages(models, reqs2[:16], 128, ref2, 1024)
        v = ref2[:, 0] != -7.0
        assert_rel(out2[v], ref2[v], TOL16, "graph replay")
        np.testing.assert_array_equal(out2[~v], -7.0)


def test_page_launch_shapes_agree_bitwise(N):
    models, reqs = _vt_setup(1, seed=62)
    reqs = reqs[:24]
    outs = []
    for shape in ((1, 4, 16), (2, 8, 8), (8, 32, 4), (1, 1, 32)):
        c = N.Context(0)
        c.set_launch(*shape)
        outs.append(_run_pages(N, c, models, reqs, 1)[0])
        c.close()
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


# ---------------------------------------------------- full-size frame + random queries
@pytest.fixture(scope="module")
def c2_model():
    return I.random_model(4096, 4096, 1024, 1024, 24, np.float16, np.float16, config=2)


def test_c2_frame_and_random_sampled(N, ctx, c2_model):
    """4096^2 atlas, T = 24, FP16 storage: the full frame through the page decoder and
    16M random queries, both at their real size, checked on the oracle subsample (2^20
    frame texels at stride 16 and the first 2^20 queries: the FP16 error's tail matters at
    this count)."""
    import torch
    m = c2_model
    dm = N.DeviceModel.from_numpy(m)
    marr = N.models_array([dm])
    t = float(I.rng(2, I.P_QUERY).random(dtype=np.float32))
    py, px = np.meshgrid(np.arange(32), np.arange(32), indexing="ij")
    rq = N.page_requests(np.zeros(1024, np.int32), px.ravel().astype(np.int32), py.ravel().astype(np.int32),
                         np.full(1024, t, np.float32), (py * 128 * 4096 + px * 128).ravel().astype(np.int64))
    nreq = torch.tensor([1024], dtype=torch.int32, device="cuda")
    # the oracle subsample: 2^20 frame texels at stride 16 and the first 2^20 random queries
    g = np.random.default_rng(21)
    sel = np.arange(0, 4096 * 4096, 16)
    xs, ys = sel % 4096, sel // 4096
    ref = O.decode_f64(m, (xs + 0.5) / 4096, (ys + 0.5) / 4096, np.full(sel.size, np.float64(np.float32(t))))
    for prec, tol in ((1, TOL16), (0, TOL32)):
        dst = torch.empty((4096 * 4096, 3), dtype=torch.float16 if prec else torch.float32, device="cuda")
        ctx.decode_pages(marr, 1, rq, nreq, 1024, 128, dst, 4096, prec)
        got = dst[torch.from_numpy(sel).cuda()].float().cpu().numpy()
        assert_rel(got, ref, tol, f"frame prec {prec}")
    q = I.uniform_queries(16_000_000, I.rng(2, I.P_QUERY, 1))
    qd = torch.from_numpy(q).cuda()
    sel = np.arange(1 << 20)
    ref = O.decode(m, q[sel])
    ws = None
    for prec, tol in ((1, TOL16), (0, TOL32)):
        out = ctx.decode(dm, qd, prec)
        got = out[torch.from_numpy(sel).cuda()].float().cpu().numpy()
        assert_rel(got, ref, tol, f"random prec {prec}")
        binned, ws = ctx.decode_binned(dm, qd, prec, workspace=ws)
        assert torch.equal(binned.view(torch.int16 if prec else torch.int32),
                           out.view(torch.int16 if prec else torch.int32)), f"binned != direct, prec {prec}"


def test_c3_vt_frame_at_real_size_and_autotuned_shape(N):
    """One frame of the virtual-texturing workload at its real size: 32 maps of side
    128 * round(2^U[1,5]) with T = 24, 2000 page requests drawn Zipf(1.1), one
    graph-replayed persistent launch at the launch shape the autotuner picks for it on this
    GPU (tile 2 x 16, 32 waves per CU); 64 texels of every request checked against the
    oracle (FP16 path)."""
    import torch
    c = N.Context(0)
    c.set_launch(2, 16, 32)
    sides = I.vt_map_sides(32, I.rng(3, I.P_MODEL))
    dms, hms = [], []
    for i, sd in enumerate(sides):
        sd = int(sd)
        m = I.random_model_torch(sd, sd, sd // 4, sd // 4, 24, seed=1000 + i, device="cuda")
        dms.append(N.DeviceModel(sd, sd, sd // 4, sd // 4, 24, m["bc4"], m["grid"], m["mlp"]))
        hms.append(m)
    marr = N.models_array(dms)
    n_req, per_row, page = 2000, 50, 128
    pitch = per_row * page
    offs = np.array([(i // per_row) * page * pitch + (i % per_row) * page for i in range(n_req)], dtype=np.int64)
    mi, px, py, t = I.vt_requests(sides, n_req, I.rng(3, I.P_REQ, 0))
    rq = N.page_requests(mi, px, py, t, offs)
    nreq = torch.tensor([n_req], dtype=torch.int32, device="cuda")
    dst = torch.full((((n_req + per_row - 1) // per_row) * page * pitch, 3), -7.0, dtype=torch.float16,
                     device="cuda")
    c.decode_pages(marr, len(dms), rq, nreq, n_req, page, dst, pitch, N.PREC_F16, graph=True)
    torch.cuda.synchronize()
    assert c.error_flags() == 0
    g = np.random.default_rng(33)
    ii, jj = g.integers(0, page, (n_req, 64)), g.integers(0, page, (n_req, 64))
    rows = offs[:, None] + jj * pitch + ii
    got = dst[torch.from_numpy(rows.ravel()).cuda()].float().cpu().numpy().reshape(n_req, 64, 3)
    for k in np.unique(mi):
        sel = np.nonzero(mi == k)[0]
        hm = hms[k]
        m = dict(W=hm["W"], H=hm["H"], Gw=hm["Gw"], Gh=hm["Gh"], T=hm["T"], bc4=hm["bc4"].cpu().numpy(),
                 grid=hm["grid"].cpu().numpy(), mlp=hm["mlp"].cpu().numpy())
        x = page * px[sel, None] + ii[sel]
        y = page * py[sel, None] + jj[sel]
        ref = O.decode_f64(m, (x.ravel() + 0.5) / m["W"], (y.ravel() + 0.5) / m["H"],
                           np.repeat(t[sel].astype(np.float64), 64))
        assert_rel(got[sel].reshape(-1, 3), ref, TOL16, f"VT map {k} (side {m['W']})")
    c.close()
