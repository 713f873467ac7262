// Decode kernels: BC4 block decoder, random-access query decode, persistent page decode.
#include "device.hpp"
#include "internal.hpp"

namespace ndgi {

// ------------------------------------------------------------------------ BC4 blocks
// IMPL selects the texel decoder: 0 the integer bc4_texel, 1 the float bc4_texel_f of the
// query, page and hybrid kernels, 2 the row decode bc4_rows of the frame and binned kernels.
template <int IMPL>
__global__ __launch_bounds__(256) void k_bc4_blocks(const uint8_t* __restrict__ blocks, int64_t n,
                                                     uint8_t* __restrict__ out) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n; b += (int64_t)gridDim.x * blockDim.x) {
    const uint2 w = ((const uint2*)blocks)[b];
    uint32_t o[4];
    if constexpr (IMPL == 2) {
      bc4_rows(w.x, w.y, 0, o[0], o[1]);
      bc4_rows(w.x, w.y, 1, o[2], o[3]);
    } else {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        uint32_t v = 0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const uint32_t t = IMPL == 1 ? (uint32_t)bc4_texel_f(w.x, w.y, 4 * r + c) : bc4_texel(w.x, w.y, 4 * r + c);
          v |= t << (8 * c);
        }
        o[r] = v;
      }
    }
    ((uint4*)out)[b] = make_uint4(o[0], o[1], o[2], o[3]);
  }
}

int launch_bc4_blocks(const uint8_t* blocks, int64_t n, uint8_t* out, int impl, hipStream_t s) {
  const int64_t want = (n + 255) / 256;
  const int grid = (int)(want < 65536 ? want : 65536);
  if (impl == 1) hipLaunchKernelGGL(k_bc4_blocks<1>, dim3(grid), dim3(256), 0, s, blocks, n, out);
  else if (impl == 2) hipLaunchKernelGGL(k_bc4_blocks<2>, dim3(grid), dim3(256), 0, s, blocks, n, out);
  else hipLaunchKernelGGL(k_bc4_blocks<0>, dim3(grid), dim3(256), 0, s, blocks, n, out);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

// ------------------------------------------------------------------- query decode
// Each wave takes passes of 64 consecutive queries (phase A: one query per lane; phase B:
// the decoder after the register handoff); 4 waves per workgroup; grid-stride.
template <int PREC, int GDT>
__global__ __launch_bounds__(256) void k_decode_query(ndgi_model m, const float* __restrict__ uvt, int64_t n,
                                                       void* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  Dec<PREC> dec;
  dec.load(m.mlp, m.mlp_dtype, lane);
  const int64_t passes = (n + 63) >> 6;
  const int64_t wave0 = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t p = wave0; p < passes; p += nwaves) {
    const int64_t mine = (p << 6) + lane;
    float u = 0.5f, v = 0.5f, t = 0.0f;
    if (mine < n) {
      u = uvt[mine * 3 + 0];
      v = uvt[mine * 3 + 1];
      t = uvt[mine * 3 + 2];
    }
    float sp[8], gr[8];
    spatial8_global(m, coord_axis(u, m.W), coord_axis(v, m.H), sp);
    query_grid8<GDT>(m, u, v, t, gr);
    const f4v acc = decode_regs<PREC>(dec, sp, gr);
    if (mine < n) store_rgb<PREC>(out, (size_t)mine, acc, !(isfinite(u) && isfinite(v) && isfinite(t)));
  }
}

int launch_decode(ndgi_ctx* ctx, const ndgi_model& m, const float* uvt, int64_t n, void* out, int prec,
                  hipStream_t s) {
  if (n == 0) return NDGI_OK;
  const int64_t passes = (n + 63) / 64;
  int64_t wgs = (passes + 3) / 4;
  const bool g16 = m.grid_dtype == NDGI_DTYPE_F16;
  const void* kern = (prec == NDGI_PREC_F16)
                         ? (g16 ? (const void*)k_decode_query<NDGI_PREC_F16, NDGI_DTYPE_F16>
                                : (const void*)k_decode_query<NDGI_PREC_F16, NDGI_DTYPE_F32>)
                         : (g16 ? (const void*)k_decode_query<NDGI_PREC_F32, NDGI_DTYPE_F16>
                                : (const void*)k_decode_query<NDGI_PREC_F32, NDGI_DTYPE_F32>);
  const int64_t cap = resident_wgs(ctx, kern);
  if (wgs > cap) wgs = cap;
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

// Global loads of one pass: this lane's BC4 block (footprint db, channel dc) and its grid
// window items (keys k0 and k1).  Issued one pass ahead of use.
struct TileLoads {
  uint2 blk;
  uint32_t g0[2], g1[2];
};

// Addressing of a sub-tile's loads: the map's block and the two keys' grid planes as uniform
// bases, and this lane's pass-invariant share (its block within a pass's four footprints and
// its two grid window items).  Offsets are 32-bit: the model check bounds the map below 4 GiB
// of blocks and the grid below 4 GiB.
// The model's buffers are device memory: global address-space pointers let each load take a
// uniform 64-bit base and a 32-bit lane offset (no 64-bit address arithmetic per lane).
typedef const __attribute__((address_space(1))) uint8_t* gbyte_ptr;
template <typename T>
__device__ __forceinline__ T gload(gbyte_ptr base, uint32_t byte_off) {
  return *(const __attribute__((address_space(1))) T*)(base + byte_off);
}
struct TileAddr {
  gbyte_ptr bc4;        // the map's blocks
  gbyte_ptr g0;         // grid of key k0: words of two FP16 channels
  gbyte_ptr g1;         // key k1
  int wb, gw, gw1, gh1;
  uint32_t boff;        // byte offset of this lane's block in a pass: footprint db, channel dc
  int nx[2], ny[2], pr[2];
};

__device__ __forceinline__ TileAddr tile_addr(const ndgi_model& m, const Keys& k, int lane, int db, int dc) {
  TileAddr a;
  const size_t plane_words = (size_t)m.Gh * m.Gw * 4;
  a.bc4 = (gbyte_ptr)m.bc4;
  a.g0 = (gbyte_ptr)m.grid + (size_t)k.k0 * plane_words * 4;
  a.g1 = (gbyte_ptr)m.grid + (size_t)k.k1 * plane_words * 4;
  a.wb = m.W >> 2;
  a.gw = m.Gw;
  a.gw1 = m.Gw - 1;
  a.gh1 = m.Gh - 1;
  a.boff = (uint32_t)(db * 64 + 8 * dc);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int item = it ? (lane < 8 ? lane + 64 : lane) : lane;   // items 64..71 on lanes 0..7
    const int n = item >> 2;
    a.pr[it] = item & 3;
    a.ny[it] = n / 6;
    a.nx[it] = n - 6 * a.ny[it];
  }
  return a;
}

// Global loads of the pass at texel (x0, y0): this lane's BC4 block and its grid window items
// of both keys (node window from grid node (x0/4 - 1, y0/4 - 1), clamped to the grid).
__device__ __forceinline__ void tile_issue(const TileAddr& a, int x0, int y0, TileLoads& t) {
  const uint32_t bi = (uint32_t)((y0 >> 2) * a.wb + (x0 >> 2)) * 64u + a.boff;
  const unsigned long long bw = gload<unsigned long long>(a.bc4, bi);
  t.blk = make_uint2((uint32_t)bw, (uint32_t)(bw >> 32));
  const int gx0 = (x0 >> 2) - 1, gy0 = (y0 >> 2) - 1;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int gx = min(max(gx0 + a.nx[it], 0), a.gw1), gy = min(max(gy0 + a.ny[it], 0), a.gh1);
    const uint32_t off = (((uint32_t)__umul24(gy, a.gw) + (uint32_t)gx) * 4u + (uint32_t)a.pr[it]) * 4u;
    t.g0[it] = gload<uint32_t>(a.g0, off);
    t.g1[it] = gload<uint32_t>(a.g1, off);
  }
}

__device__ __forceinline__ float2 half2_bits(uint32_t w) {
  return make_float2((float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu)),
                     (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16)));
}

// FP16-grid tile path over one sub-tile.  Passes run row-slab by column-slab; the loads of
// pass p+1 are in flight while pass p computes.
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
  const int bx = page * rq.page_x + ox, by = page * rq.page_y + oy;
  const int np = tw * th;
  const TileAddr ta = tile_addr(m, k, lane, db, dc);
  // this lane's output texel (row g, column j) of the sub-tile's first pass; later passes add
  // a uniform offset
  _Float16* const out0 = (_Float16*)dst + (rq.dst_offset + (int64_t)(oy + g) * pitch + (ox + j)) * 3;
  TileLoads cur;
  tile_issue(ta, bx, by, cur);
  for (int p = 0; p < np; ++p) {
    const int a = p % tw, b = p / tw;
    // stage this pass: time-blend the grid window, decode the BC4 rows
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      if (it == 0 || lane < 8) {
        const float2 v0 = half2_bits(cur.g0[it]), v1 = half2_bits(cur.g1[it]);
        // w0 v0 as an FMA with a zero addend: one mixed-precision FMA on the FP16 word (the
        // same rounded product)
        L.gt[it ? lane + 64 : lane] =
            make_float2(fmaf(k.w1, v1.x, fmaf(k.w0, v0.x, 0.0f)), fmaf(k.w1, v1.y, fmaf(k.w0, v0.y, 0.0f)));
      }
    }
    uint32_t row0, row1;
    bc4_rows(cur.blk.x, cur.blk.y, drp, row0, row1);
    L.sp[dc * 20 + (2 * drp) * 4 + db] = row0;
    L.sp[dc * 20 + (2 * drp + 1) * 4 + db] = row1;
    if (p + 1 < np) {
      const int a1 = (p + 1) % tw, b1 = (p + 1) / tw;
      tile_issue(ta, bx + 16 * a1, by + 4 * b1, cur);
    }
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
    store_rgb<NDGI_PREC_F16>(out0 + ((int64_t)(4 * b) * pitch + 16 * a) * 3, 0, acc, false);
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

// Maps the FP16 tile kernel serves: grid at a quarter of the texel resolution, FP16 grid
// and decoder.
__device__ __forceinline__ bool tile_eligible(const ndgi_model& m) {
  return m.W == 4 * m.Gw && m.H == 4 * m.Gh && m.grid_dtype == NDGI_DTYPE_F16 && m.mlp_dtype == NDGI_DTYPE_F16;
}

// Request scan shared by the two page kernels: item `it` -> request, sub-tile, model.
// Returns false (and flags the request once) when the request is invalid.
struct PageItem {
  ndgi_page_req rq;
  int s;
};

__device__ __forceinline__ bool page_item(const ndgi_model* __restrict__ models, int32_t n_models,
                                          const ndgi_page_req* __restrict__ reqs, int64_t it, int64_t per_req,
                                          int page, int lane, int& cur, ndgi_model& m, PageItem& pi,
                                          uint32_t* __restrict__ flags, bool report) {
  const int r = (int)(it / per_req);
  pi.s = (int)(it - (int64_t)r * per_req);
  pi.rq = reqs[r];
  const ndgi_page_req& rq = pi.rq;
  bool ok = rq.model >= 0 && rq.model < n_models && rq.page_x >= 0 && rq.page_y >= 0;
  if (ok && rq.model != cur) {
    m = models[rq.model];
    cur = rq.model;
  }
  ok = ok && (int64_t)page * (rq.page_x + 1) <= m.W && (int64_t)page * (rq.page_y + 1) <= m.H;
  if (!ok && report && lane == 0 && pi.s == 0) atomicOr(flags, NDGI_FLAG_BAD_PAGE_REQUEST);
  return ok;
}

// FP16 requests on tile-eligible maps (tile path).
__global__ __launch_bounds__(256) void k_decode_tiles(const ndgi_model* __restrict__ models, int32_t n_models,
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
  Dec16 dec;
  int dmodel = -1, cur = -1;
  ndgi_model m = {};
  PageItem pi;
  for (int64_t it = wave0; it < total; it += nwaves) {
    if (!page_item(models, n_models, reqs, it, per_req, page, lane, cur, m, pi, flags, true)) continue;
    if (!tile_eligible(m)) continue;                            // served by the general kernel
    if (dmodel != pi.rq.model) {
      load_dec16<NDGI_DTYPE_F16, true>(dec, m.mlp, lane);
      dmodel = pi.rq.model;
    }
    const Keys k = make_keys(pi.rq.t, m.T);
    const int ox = (pi.s % nsx) * sub_w, oy = (pi.s / nsx) * sub_h;
    tile_subtile(dec, m, pi.rq, k, page, ox, oy, tw, th, dst, pitch, lane, tlds[threadIdx.x >> 6]);
  }
}

// General page decode (any grid ratio, either precision).  With SKIP_TILES the requests the
// tile kernel serves are skipped.
template <int PREC, bool SKIP_TILES>
__global__ __launch_bounds__(256) void k_decode_pages(const ndgi_model* __restrict__ models, int32_t n_models,
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
  Dec<PREC> dec;
  int dmodel = -1, cur = -1;
  ndgi_model m = {};
  PageItem pi;
  for (int64_t it = wave0; it < total; it += nwaves) {
    // the tile kernel already reported invalid requests when it runs
    if (!page_item(models, n_models, reqs, it, per_req, page, lane, cur, m, pi, flags, !SKIP_TILES)) continue;
    const bool r4 = m.W == 4 * m.Gw && m.H == 4 * m.Gh;
    if (SKIP_TILES && tile_eligible(m)) continue;
    if (dmodel != pi.rq.model) {
      dec.load(m.mlp, m.mlp_dtype, lane);
      dmodel = pi.rq.model;
    }
    const Keys k = make_keys(pi.rq.t, m.T);
    const int ox = (pi.s % nsx) * sub_w, oy = (pi.s / nsx) * sub_h;
    if (m.grid_dtype == NDGI_DTYPE_F16) {
      if (r4) page_subtile<PREC, NDGI_DTYPE_F16, true>(dec, m, pi.rq, k, page, ox, oy, tw, th, dst, pitch, lane);
      else page_subtile<PREC, NDGI_DTYPE_F16, false>(dec, m, pi.rq, k, page, ox, oy, tw, th, dst, pitch, lane);
    } else {
      if (r4) page_subtile<PREC, NDGI_DTYPE_F32, true>(dec, m, pi.rq, k, page, ox, oy, tw, th, dst, pitch, lane);
      else page_subtile<PREC, NDGI_DTYPE_F32, false>(dec, m, pi.rq, k, page, ox, oy, tw, th, dst, pitch, lane);
    }
  }
}

int launch_pages(ndgi_ctx* ctx, const ndgi_model* models, int32_t n_models, const ndgi_page_req* reqs,
                 const int32_t* n_reqs, int32_t max_reqs, int32_t page, void* dst, int64_t pitch, int prec,
                 hipStream_t s) {
  if (prec == NDGI_PREC_F16) {
    hipLaunchKernelGGL(k_decode_tiles, dim3(resident_wgs(ctx, (const void*)k_decode_tiles)), dim3(256), 0, s, models,
                       n_models, reqs, n_reqs, max_reqs, page, dst, pitch, ctx->tile_w, ctx->tile_h, ctx->flags_dev);
    hipLaunchKernelGGL((k_decode_pages<NDGI_PREC_F16, true>),
                       dim3(resident_wgs(ctx, (const void*)k_decode_pages<NDGI_PREC_F16, true>)), dim3(256), 0, s,
                       models, n_models, reqs, n_reqs, max_reqs, page, dst, pitch, ctx->tile_w, ctx->tile_h,
                       ctx->flags_dev);
  } else {
    hipLaunchKernelGGL((k_decode_pages<NDGI_PREC_F32, false>),
                       dim3(resident_wgs(ctx, (const void*)k_decode_pages<NDGI_PREC_F32, false>)), dim3(256), 0, s,
                       models, n_models, reqs, n_reqs, max_reqs, page, dst, pitch, ctx->tile_w, ctx->tile_h,
                       ctx->flags_dev);
  }
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

}  // namespace ndgi
