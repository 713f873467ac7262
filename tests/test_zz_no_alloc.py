"""The allocation-free binned decode (static device scratch) against the binned decode with
a caller workspace, through the C ABI: bit for bit, on two calls in a row (the second with
fewer queries and another map, so stale scratch from the first must not leak), and the
size limit refused on the host before any launch."""
import ctypes

import numpy as np
import pytest

from oracle import ndgi_oracle as O
from paper_2604_12625_amd import inputs as I
from tests.gpu_util import assert_rel, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    torch = torch_cuda()
    from paper_2604_12625_amd import ndgi as N
    ctx = N.Context(0)
    yield torch, N, ctx
    ctx.close()


def _both(torch, N, ctx, model, q, prec):
    dm = N.DeviceModel.from_numpy(model)
    uvt = torch.from_numpy(q).cuda()
    ref, _ = ctx.decode_binned(dm, uvt, prec)
    out = torch.full_like(ref, float("nan"))
    ctx.decode_binned_noalloc(dm, uvt, out, prec)
    torch.cuda.synchronize()
    return out.float().cpu().numpy(), ref.float().cpu().numpy()


@pytest.mark.parametrize("prec,tol", [(1, 2e-3), (0, 1e-5)])
def test_noalloc_equals_workspace_binned_on_two_calls(env, prec, tol):
    torch, N, ctx = env
    # call 1: a 1024^2 map with a 256^2 x 24 grid (grid-aligned bins), 1.5M queries
    m1 = I.random_model(1024, 1024, 256, 256, 24, np.float16, np.float16, config=70)
    q1 = I.uniform_queries(1_500_000, I.rng(70, I.P_QUERY, prec))
    got, ref = _both(torch, N, ctx, m1, q1, prec)
    np.testing.assert_array_equal(got, ref)
    sel = np.random.default_rng(70).integers(0, q1.shape[0], 2048)
    assert_rel(got[sel], O.decode(m1, q1[sel]), tol, "noalloc call 1")
    # call 2: fewer queries on a ragged 200 x 148 map binned by texel tiles
    m2 = I.random_model(200, 148, 70, 30, 12, np.float16, np.float16, config=71)
    q2 = np.concatenate([I.uniform_queries(30001, I.rng(71, I.P_QUERY, prec)),
                         I.texel_centre_queries(200, 148, [0.61])])
    got, ref = _both(torch, N, ctx, m2, q2, prec)
    np.testing.assert_array_equal(got, ref)
    assert_rel(got, O.decode(m2, q2), tol, "noalloc call 2")


def test_noalloc_refuses_more_queries_than_its_scratch_holds(env):
    torch, N, ctx = env
    m = I.random_model(1024, 1024, 256, 256, 24, np.float16, np.float16, config=72)
    dm = N.DeviceModel.from_numpy(m)
    n_max = 4_061_680            # the largest batch whose layout fits 64 MiB on this map
    need = ctypes.c_int64()
    assert N.lib().ndgi_decode_binned_workspace(ctypes.byref(dm.desc), n_max, ctypes.byref(need)) == N.OK
    assert need.value <= 64 << 20
    assert N.lib().ndgi_decode_binned_workspace(ctypes.byref(dm.desc), n_max + 1, ctypes.byref(need)) == N.OK
    assert need.value > 64 << 20
    # refused on the host from n alone, before any launch (the buffers are never read)
    uvt = torch.zeros((4, 3), dtype=torch.float32, device="cuda")
    out = torch.zeros((4, 3), dtype=torch.float16, device="cuda")
    rc = N.lib().ndgi_decode_binned_noalloc(ctx.h, ctypes.byref(dm.desc), ctypes.c_void_p(uvt.data_ptr()),
                                            n_max + 1, ctypes.c_void_p(out.data_ptr()), 1, None)
    assert rc == N.ERR_INVALID_ARG
    assert b"static" in N.lib().ndgi_last_error()
    # n = 0 is a no-op
    assert N.lib().ndgi_decode_binned_noalloc(ctx.h, ctypes.byref(dm.desc), None, 0, None, 1, None) == N.OK
