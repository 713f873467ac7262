// Decode kernels: BC4 block decoder, random-access query decode, persistent page decode.
#include "device.hpp"
#include "internal.hpp"

namespace ndgi {

// ------------------------------------------------------------------------ BC4 blocks
__global__ __launch_bounds__(256) void k_bc4_blocks(const uint8_t* __restrict__ blocks, int64_t n,
                                                     uint8_t* __restrict__ out) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n; b += (int64_t)gridDim.x * blockDim.x) {
    const uint2 w = ((const uint2*)blocks)[b];
    uint32_t o[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      uint32_t v = 0;
#pragma unroll
      for (int c = 0; c < 4; ++c) v |= bc4_texel(w.x, w.y, 4 * r + c) << (8 * c);
      o[r] = v;
    }
    ((uint4*)out)[b] = make_uint4(o[0], o[1], o[2], o[3]);
  }
}

int launch_bc4_blocks(const uint8_t* blocks, int64_t n, uint8_t* out, hipStream_t s) {
  const int64_t want = (n + 255) / 256;
  const int grid = (int)(want < 65536 ? want : 65536);
  hipLaunchKernelGGL(k_bc4_blocks, dim3(grid), dim3(256), 0, s, blocks, n, out);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

// ------------------------------------------------------------------- query decode
// Each wave takes passes of 64 consecutive queries; 4 waves per workgroup; grid-stride.
template <int PREC>
__global__ __launch_bounds__(256) void k_decode_query(ndgi_model m, const float* __restrict__ uvt, int64_t n,
                                                       void* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, j = lane & 15;
  Dec<PREC> dec;
  dec.load(m.mlp, m.mlp_dtype, lane);
  const int64_t passes = (n + 63) >> 6;
  const int64_t wave0 = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t p = wave0; p < passes; p += nwaves) {
    f4v acc = dec.bias3();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t idx = (p << 6) + 16 * q + j;
      float u = 0.5f, v = 0.5f, t = 0.0f;
      if (idx < n) {
        u = uvt[idx * 3 + 0];
        v = uvt[idx * 3 + 1];
        t = uvt[idx * 3 + 2];
      }
      float f[4];
      query_inputs(m, u, v, t, g, f);
      dec.group(f, q, acc);
    }
    const int64_t mine = (p << 6) + lane;
    if (mine < n) {
      const float u = uvt[mine * 3 + 0], v = uvt[mine * 3 + 1], t = uvt[mine * 3 + 2];
      const bool bad = !(isfinite(u) && isfinite(v) && isfinite(t));
      store_rgb<PREC>(out, (size_t)mine, acc, bad);
    }
  }
}

int launch_decode(ndgi_ctx* ctx, const ndgi_model& m, const float* uvt, int64_t n, void* out, int prec,
                  hipStream_t s) {
  if (n == 0) return NDGI_OK;
  const int64_t passes = (n + 63) / 64;
  int64_t wgs = (passes + 3) / 4;
  const int64_t cap = (int64_t)ctx->n_cu * (ctx->waves_per_cu > 4 ? ctx->waves_per_cu / 4 : 1);
  if (wgs > cap) wgs = cap;
  if (prec == NDGI_PREC_F16)
    hipLaunchKernelGGL(k_decode_query<NDGI_PREC_F16>, dim3((unsigned)wgs), dim3(256), 0, s, m, uvt, n, out);
  else
    hipLaunchKernelGGL(k_decode_query<NDGI_PREC_F32>, dim3((unsigned)wgs), dim3(256), 0, s, m, uvt, n, out);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

// -------------------------------------------------------------- persistent page decode
// Work item = (request, sub-tile of 16*tw x 4*th texels).  Every wave of the persistent
// grid takes items round-robin (items cost the same, so a static schedule balances
// without a shared counter); a pass covers 16 columns x 4 rows: group q is row q.
template <int PREC>
__global__ __launch_bounds__(256) void k_decode_pages(const ndgi_model* __restrict__ models, int32_t n_models,
                                                       const ndgi_page_req* __restrict__ reqs,
                                                       const int32_t* __restrict__ n_reqs_dev, int32_t max_reqs,
                                                       int32_t page, void* __restrict__ dst, int64_t pitch, int tw,
                                                       int th, uint32_t* __restrict__ flags) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, j = lane & 15;
  int n_req = *n_reqs_dev;
  n_req = n_req < 0 ? 0 : (n_req > max_reqs ? max_reqs : n_req);
  const int sub_w = 16 * tw, sub_h = 4 * th;
  const int nsx = page / sub_w, nsy = page / sub_h;
  const int64_t per_req = (int64_t)nsx * nsy;
  const int64_t total = (int64_t)n_req * per_req;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t wave0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));

  Dec<PREC> dec;
  int cur = -1;
  ndgi_model m = {};
  for (int64_t it = wave0; it < total; it += nwaves) {
    const int r = (int)(it / per_req);
    const int s = (int)(it - (int64_t)r * per_req);
    const ndgi_page_req rq = reqs[r];
    bool ok = rq.model >= 0 && rq.model < n_models && rq.page_x >= 0 && rq.page_y >= 0;
    if (ok && rq.model != cur) {
      m = models[rq.model];
      cur = rq.model;
      dec.load(m.mlp, m.mlp_dtype, lane);
    }
    ok = ok && (int64_t)page * (rq.page_x + 1) <= m.W && (int64_t)page * (rq.page_y + 1) <= m.H;
    if (!ok) {
      if (lane == 0 && s == 0) atomicOr(flags, NDGI_FLAG_BAD_PAGE_REQUEST);
      continue;
    }
    const Keys k = make_keys(rq.t, m.T);
    const int ox = (s % nsx) * sub_w, oy = (s / nsx) * sub_h;   // sub-tile origin in the page
    const int bx = page * rq.page_x, by = page * rq.page_y;
    for (int b = 0; b < th; ++b) {
      for (int a = 0; a < tw; ++a) {
        f4v acc = dec.bias3();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float f[4];
          texel_inputs(m, bx + ox + 16 * a + j, by + oy + 4 * b + q, k, g, f);
          dec.group(f, q, acc);
        }
        // lane (g, j) holds the texel of row g of this pass
        const int64_t di = rq.dst_offset + (int64_t)(oy + 4 * b + g) * pitch + (ox + 16 * a + j);
        store_rgb<PREC>(dst, (size_t)di, acc, false);
      }
    }
  }
}

int launch_pages(ndgi_ctx* ctx, const ndgi_model* models, int32_t n_models, const ndgi_page_req* reqs,
                 const int32_t* n_reqs, int32_t max_reqs, int32_t page, void* dst, int64_t pitch, int prec,
                 hipStream_t s) {
  const int wgs = ctx->n_cu * ctx->waves_per_cu / 4 > 0 ? ctx->n_cu * ctx->waves_per_cu / 4 : 1;
  if (prec == NDGI_PREC_F16)
    hipLaunchKernelGGL(k_decode_pages<NDGI_PREC_F16>, dim3(wgs), dim3(256), 0, s, models, n_models, reqs, n_reqs,
                       max_reqs, page, dst, pitch, ctx->tile_w, ctx->tile_h, ctx->flags_dev);
  else
    hipLaunchKernelGGL(k_decode_pages<NDGI_PREC_F32>, dim3(wgs), dim3(256), 0, s, models, n_models, reqs, n_reqs,
                       max_reqs, page, dst, pitch, ctx->tile_w, ctx->tile_h, ctx->flags_dev);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

}  // namespace ndgi
