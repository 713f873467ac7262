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
template <int PREC, int GDT>
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
      query_inputs<GDT>(m, u, v, t, g, f);
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
  const bool g16 = m.grid_dtype == NDGI_DTYPE_F16;
  if (prec == NDGI_PREC_F16 && g16)
    hipLaunchKernelGGL((k_decode_query<NDGI_PREC_F16, NDGI_DTYPE_F16>), dim3((unsigned)wgs), dim3(256), 0, s, m, uvt, n, out);
  else if (prec == NDGI_PREC_F16)
    hipLaunchKernelGGL((k_decode_query<NDGI_PREC_F16, NDGI_DTYPE_F32>), dim3((unsigned)wgs), dim3(256), 0, s, m, uvt, n, out);
  else if (g16)
    hipLaunchKernelGGL((k_decode_query<NDGI_PREC_F32, NDGI_DTYPE_F16>), dim3((unsigned)wgs), dim3(256), 0, s, m, uvt, n, out);
  else
    hipLaunchKernelGGL((k_decode_query<NDGI_PREC_F32, NDGI_DTYPE_F32>), dim3((unsigned)wgs), dim3(256), 0, s, m, uvt, n, out);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

// -------------------------------------------------------------- persistent page decode
// Work item = (request, sub-tile of 16*tw x 4*th texels).  Every wave of the persistent
// grid takes items round-robin (items cost the same, so a static schedule balances
// without a shared counter); a pass covers 16 columns x 4 rows: group q is row q.
// ------------------------------------------------------------ texel-centre tile path
// Used for FP16 decode of maps whose grid is a quarter of the texel resolution.  A pass
// is 16 columns x 4 rows = exactly four 4x4 BC4 footprints.  The wave first decodes the
// 4 footprints x 8 channels cooperatively (lane = footprint, channel, row pair) into LDS
// and interpolates the grid window of the pass (6 x 3 nodes) in time into LDS; then each
// group (one row) reads its lane share and runs the decoder.

struct TileLds {
  uint32_t sp[8 * 20];   // decoded bytes [channel][row][16 columns]; channel stride 80 B
                         // keeps the four lane groups of a read on distinct banks
  float2 gt[18 * 4];     // [node row 0..2][node column 0..5][channel pair], time-blended
};

// Rows 2rp and 2rp+1 of a BC4 block (lo = bytes 0..3, hi = bytes 4..7) as 4 bytes each.
// The 8-entry palette is built once: the interior entries are 1024 + e0 + 0.5 + j*(e1-e0)/D
// rounded toward zero to FP16 (integers are exact in [1024, 2048)), which equals the
// palette's round-to-nearest value since the exact quotient is never within 0.5/D of an
// integer.  The row's four 3-bit selectors are spread into a byte selector and one
// v_perm_b32 picks four texels from the palette.
__device__ __forceinline__ void bc4_rows(uint32_t lo, uint32_t hi, int rp, uint32_t& r0, uint32_t& r1) {
  const uint32_t ie0 = lo & 0xffu, ie1 = (lo >> 8) & 0xffu;
  const bool eight = ie0 > ie1;
  const float e0 = (float)ie0, e1 = (float)ie1;
  const float B = (e1 - e0) * (eight ? (1.0f / 7.0f) : 0.2f);
  const float A = e0 + 1024.5f;
  const uint32_t p12 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(fmaf(1.0f, B, A), fmaf(2.0f, B, A)));
  const uint32_t p34 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(fmaf(3.0f, B, A), fmaf(4.0f, B, A)));
  const uint32_t p56 = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(fmaf(5.0f, B, A), fmaf(6.0f, B, A)));
  // palette bytes: [e0, e1, p1, p2 | p3, p4, p5, p6] or, in 6-value mode, [.. | p3, p4, 0, 255]
  const uint32_t pal_lo = __builtin_amdgcn_perm(p12, lo, 0x06040100u);
  const uint32_t pal_hi = __builtin_amdgcn_perm(p56, p34, eight ? 0x06040200u : 0x0D0C0200u);
  const uint64_t bits = (((uint64_t)hi << 32) | lo) >> (16 + 24 * rp);
  const uint32_t c24 = (uint32_t)bits;
#pragma unroll
  for (int rr = 0; rr < 2; ++rr) {
    const uint32_t c = (c24 >> (12 * rr)) & 0xfffu;    // four 3-bit selectors
    uint32_t t = (c | (c << 10)) & 0x003f003fu;
    t = (t | (t << 5)) & 0x07070707u;                  // one selector per byte
    const uint32_t v = __builtin_amdgcn_perm(pal_hi, pal_lo, t);
    if (rr == 0) r0 = v;
    else r1 = v;
  }
}

template <int GDT>
__device__ __forceinline__ void tile_subtile(const Dec16& dec, const ndgi_model& m, const ndgi_page_req& rq,
                                             const Keys& k, int page, int ox, int oy, int tw, int th, void* dst,
                                             int64_t pitch, int lane, TileLds& L) {
  const int g = lane >> 4, j = lane & 15;
  // grid corner of this lane's column in the node window, and its weight (x % 4 = j % 4)
  const int cx = ((2 * j - 3) >> 3) + 1;
  const float wx1 = (float)((2 * j - 3) & 7) * 0.125f, wx0 = 1.0f - wx1;
  // decode role: footprint db, channel dc, row pair drp
  const int db = lane >> 4, dc = (lane >> 1) & 7, drp = lane & 1;
  const uint8_t* sp8 = (const uint8_t*)L.sp;
  const int bx = page * rq.page_x, by = page * rq.page_y;
  for (int b = 0; b < th; ++b) {
    for (int a = 0; a < tw; ++a) {
      const int x0 = bx + ox + 16 * a, y0 = by + oy + 4 * b;
      const uint2 blk = *(const uint2*)(m.bc4 + ((size_t)(y0 >> 2) * (m.W >> 2) + (x0 >> 2) + db) * 64 + 8 * dc);
      // grid window: 18 nodes x 4 channel pairs, clamped to the grid, blended in time
      const int gx0 = (x0 >> 2) - 1, gy0 = (y0 >> 2) - 1;
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const int item = lane + 64 * it;
        if (item < 72) {
          const int n = item >> 2, pr = item & 3;
          const int ny = n / 6, nx = n - 6 * ny;
          const int gx = min(max(gx0 + nx, 0), m.Gw - 1), gy = min(max(gy0 + ny, 0), m.Gh - 1);
          const size_t node = (size_t)gy * m.Gw + gx;
          const size_t plane = (size_t)m.Gh * m.Gw;
          const float2 v0 = grid_pair<GDT>(m.grid, (size_t)k.k0 * plane + node, pr);
          const float2 v1 = grid_pair<GDT>(m.grid, (size_t)k.k1 * plane + node, pr);
          L.gt[item] = make_float2(fmaf(k.w1, v1.x, k.w0 * v0.x), fmaf(k.w1, v1.y, k.w0 * v0.y));
        }
      }
      uint32_t row0, row1;
      bc4_rows(blk.x, blk.y, drp, row0, row1);
      L.sp[dc * 20 + (2 * drp) * 4 + db] = row0;
      L.sp[dc * 20 + (2 * drp + 1) * 4 + db] = row1;
      wave_sync();
      f4v acc = dec.c3;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t sa = sp8[(2 * g) * 80 + q * 16 + j];
        const uint32_t sb = sp8[(2 * g + 1) * 80 + q * 16 + j];
        const uint32_t spair = sa | (sb << 16) | 0x64006400u;
        const int cy = ((2 * q - 3) >> 3) + 1;
        const float wy1 = (float)((2 * q - 3) & 7) * 0.125f, wy0 = 1.0f - wy1;
        const float2 c00 = L.gt[(cy * 6 + cx) * 4 + g], c01 = L.gt[(cy * 6 + cx + 1) * 4 + g];
        const float2 c10 = L.gt[((cy + 1) * 6 + cx) * 4 + g], c11 = L.gt[((cy + 1) * 6 + cx + 1) * 4 + g];
        const float ga = wy0 * fmaf(wx1, c01.x, wx0 * c00.x) + wy1 * fmaf(wx1, c11.x, wx0 * c10.x);
        const float gb = wy0 * fmaf(wx1, c01.y, wx0 * c00.y) + wy1 * fmaf(wx1, c11.y, wx0 * c10.y);
        dec16_group(dec, texel_x(spair, ga, gb), q, acc);
      }
      wave_sync();
      const int64_t di = rq.dst_offset + (int64_t)(oy + 4 * b + g) * pitch + (ox + 16 * a + j);
      store_rgb<NDGI_PREC_F16>(dst, (size_t)di, acc, false);
    }
  }
}

// Decode one (16*tw) x (4*th) sub-tile of a page; a pass covers 16 columns x 4 rows and
// group q of the pass is row q.
template <int PREC, int GDT, bool R4>
__device__ __forceinline__ void page_subtile(const Dec<PREC>& dec, const ndgi_model& m, const ndgi_page_req& rq,
                                             const Keys& k, int page, int ox, int oy, int tw, int th, void* dst,
                                             int64_t pitch, int lane) {
  const int g = lane >> 4, j = lane & 15;
  const int bx = page * rq.page_x, by = page * rq.page_y;
  for (int b = 0; b < th; ++b) {
    for (int a = 0; a < tw; ++a) {
      f4v acc = dec.bias3();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float f[4];
        texel_inputs<GDT, R4>(m, bx + ox + 16 * a + j, by + oy + 4 * b + q, k, g, f);
        dec.group(f, q, acc);
      }
      // lane (g, j) holds the texel of row g of this pass
      const int64_t di = rq.dst_offset + (int64_t)(oy + 4 * b + g) * pitch + (ox + 16 * a + j);
      store_rgb<PREC>(dst, (size_t)di, acc, false);
    }
  }
}

template <int PREC>
__global__ __launch_bounds__(256, 2) void k_decode_pages(const ndgi_model* __restrict__ models, int32_t n_models,
                                                          const ndgi_page_req* __restrict__ reqs,
                                                          const int32_t* __restrict__ n_reqs_dev, int32_t max_reqs,
                                                          int32_t page, void* __restrict__ dst, int64_t pitch, int tw,
                                                          int th, uint32_t* __restrict__ flags) {
  const int lane = threadIdx.x & 63;
  int n_req = *n_reqs_dev;
  n_req = n_req < 0 ? 0 : (n_req > max_reqs ? max_reqs : n_req);
  const int sub_w = 16 * tw, sub_h = 4 * th;
  const int nsx = page / sub_w, nsy = page / sub_h;
  const int64_t per_req = (int64_t)nsx * nsy;
  const int64_t total = (int64_t)n_req * per_req;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int64_t wave0 = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  __shared__ TileLds tlds[4];

  // one decoder in registers, reloaded when the model or its form changes
  Dec<PREC> dec;
  int dmodel = -1, dform = -1;   // form 0: general inputs, 1: texel-centre (tile) inputs
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
    }
    ok = ok && (int64_t)page * (rq.page_x + 1) <= m.W && (int64_t)page * (rq.page_y + 1) <= m.H;
    if (!ok) {
      if (lane == 0 && s == 0) atomicOr(flags, NDGI_FLAG_BAD_PAGE_REQUEST);
      continue;
    }
    const Keys k = make_keys(rq.t, m.T);
    const int ox = (s % nsx) * sub_w, oy = (s / nsx) * sub_h;   // sub-tile origin in the page
    const bool r4 = m.W == 4 * m.Gw && m.H == 4 * m.Gh;
    const int form = (PREC == NDGI_PREC_F16 && r4) ? 1 : 0;
    if (dmodel != rq.model || dform != form) {
      if constexpr (PREC == NDGI_PREC_F16) {
        if (form) {
          if (m.mlp_dtype == NDGI_DTYPE_F16) load_dec16<NDGI_DTYPE_F16, true>(dec.d, m.mlp, lane);
          else load_dec16<NDGI_DTYPE_F32, true>(dec.d, m.mlp, lane);
        } else {
          dec.load(m.mlp, m.mlp_dtype, lane);
        }
      } else {
        dec.load(m.mlp, m.mlp_dtype, lane);
      }
      dmodel = rq.model;
      dform = form;
    }
    if constexpr (PREC == NDGI_PREC_F16) {
      if (form) {
        if (m.grid_dtype == NDGI_DTYPE_F16)
          tile_subtile<NDGI_DTYPE_F16>(dec.d, m, rq, k, page, ox, oy, tw, th, dst, pitch, lane, tlds[threadIdx.x >> 6]);
        else
          tile_subtile<NDGI_DTYPE_F32>(dec.d, m, rq, k, page, ox, oy, tw, th, dst, pitch, lane, tlds[threadIdx.x >> 6]);
        continue;
      }
    }
    if (m.grid_dtype == NDGI_DTYPE_F16) {
      if (r4) page_subtile<PREC, NDGI_DTYPE_F16, true>(dec, m, rq, k, page, ox, oy, tw, th, dst, pitch, lane);
      else page_subtile<PREC, NDGI_DTYPE_F16, false>(dec, m, rq, k, page, ox, oy, tw, th, dst, pitch, lane);
    } else {
      if (r4) page_subtile<PREC, NDGI_DTYPE_F32, true>(dec, m, rq, k, page, ox, oy, tw, th, dst, pitch, lane);
      else page_subtile<PREC, NDGI_DTYPE_F32, false>(dec, m, rq, k, page, ox, oy, tw, th, dst, pitch, lane);
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
