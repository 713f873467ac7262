// Device building blocks of the NDGI decode path on gfx950 (wave64, CDNA4 MFMA).
//
// Work layout of the decoder (used by every decode kernel):
//   A wave decodes 64 texels per pass, as 4 groups of 16.  For group q, lane
//   (g = lane/16, j = lane%16) computes four decoder inputs of texel 16q+j:
//   spatial channels 2g, 2g+1 and grid channels 2g, 2g+1.  Those four values are
//   exactly the lane's share of the B operand of a 16x16xK MFMA with the 16 texels as
//   columns, so the feature stage needs no cross-lane exchange.  The MLP runs as
//   D = W x with hidden units as rows: the C layout of one layer (lane holds rows
//   4g..4g+3 of column j) is again the lane's K share of the next layer's B operand.
//   The K order this induces is folded into the weights once per model.  The output
//   layer of the 4 groups accumulates into one 16x16 tile whose rows 4q..4q+2 hold
//   group q, so after 4 groups lane l owns the RGB of texel l of the pass.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "ndgi.h"

namespace ndgi {

typedef _Float16 h4v __attribute__((ext_vector_type(4)));
typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

// packed decoder parameters [W1 32x16 | b1 | W2 32x32 | b2 | W3 3x32 | b3]
constexpr int kOffW1 = 0, kOffB1 = 512, kOffW2 = 544, kOffB2 = 1568, kOffW3 = 1600, kOffB3 = 1696;

template <int DT>
__device__ __forceinline__ float ld(const void* p, size_t i) {
  if constexpr (DT == NDGI_DTYPE_F16) return (float)((const _Float16*)p)[i];
  else return ((const float*)p)[i];
}

// Decoder input fed by element e (0..3) of lane group g in the first layer:
// spatial 2g, 2g+1, grid 2g, 2g+1 (inputs are ordered [S0..S7, G0..G7]).
__device__ __forceinline__ int input_of(int g, int e) { return e < 2 ? 2 * g + e : 8 + 2 * g + (e - 2); }
// Hidden unit fed by element e (0..7) of lane group g in a 32-deep K operand: the
// lane's rows 4g..4g+3 of the first and of the second 16-row output tile.
__device__ __forceinline__ int unit_of(int g, int e) { return e < 4 ? 4 * g + e : 16 + 4 * g + (e - 4); }

// Order LDS traffic of one wave: writes before the barrier are visible to reads after it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------------ BC4 texel
// 8-byte block: e0, e1, then a 48-bit little-endian selector field; texel s uses bits
// 3s..3s+2.  lo = bytes 0..3, hi = bytes 4..7.  Value: selector 0 -> e0, 1 -> e1;
// e0 > e1: interior selector c -> round(((7-j) e0 + j e1)/7), j = c-1; otherwise
// round(((5-j) e0 + j e1)/5) for c = 2..5, and 0 / 255 for c = 6 / 7.
__device__ __forceinline__ uint32_t bc4_texel(uint32_t lo, uint32_t hi, uint32_t slot) {
  const uint32_t e0 = lo & 0xffu, e1 = (lo >> 8) & 0xffu;
  const uint64_t sel = ((uint64_t)hi << 16) | (uint64_t)(lo >> 16);
  const uint32_t c = (uint32_t)(sel >> (3u * slot)) & 7u;
  const bool eight = e0 > e1;
  // j: 0 selects e0, the top value selects e1, interior codes step in between
  const uint32_t top = eight ? 7u : 5u;
  const uint32_t j = c == 0u ? 0u : (c == 1u ? top : c - 1u);
  uint32_t v;
  if (eight) {
    v = ((7u - j) * e0 + j * e1 + 3u) / 7u;
  } else {
    const uint32_t jj = j > 5u ? 5u : j;
    v = ((5u - jj) * e0 + jj * e1 + 2u) / 5u;
    if (c >= 6u) v = (c == 6u) ? 0u : 255u;
  }
  return v;
}

// Same value as bc4_texel, as a float, with no integer division: for selector c the
// palette entry is floor(e0 + 0.5 + j (e1 - e0) / D) with D = 7 (e0 > e1) or 5, and
// j = 0 for c = 0, D for c = 1, c - 1 otherwise (the exact quotient is never within 0.5/D
// of an integer, so the rounded FMA floors correctly); in 6-value mode c = 6, 7 give 0, 255.
__device__ __forceinline__ float bc4_texel_f(uint32_t lo, uint32_t hi, uint32_t slot) {
  const float e0 = (float)(lo & 0xffu), e1 = (float)((lo >> 8) & 0xffu);
  const bool eight = e0 > e1;
  const float B = (e1 - e0) * (eight ? (1.0f / 7.0f) : 0.2f);
  const uint32_t code = (uint32_t)((((uint64_t)hi << 32) | lo) >> (16u + 3u * slot)) & 7u;
  const uint32_t lut = eight ? 0x65432170u : 0x00432150u;
  const float jf = (float)((lut >> (4u * code)) & 15u);
  float v = floorf(fmaf(jf, B, e0 + 0.5f));
  if (!eight && code >= 6u) v = (code == 7u) ? 255.0f : 0.0f;
  return v;
}

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

// ------------------------------------------------------------------ sampling helpers
struct Axis { int i0, i1; float w0, w1; };

// Axis of normalised coordinate c with the texel-centre convention: continuous position
// c*size - 0.5, neighbours floor() and floor()+1 clamped to [0, size-1].  The cell and the
// fraction come from the exact product: the fraction is one fused multiply-add,
// c*size - 0.5 - floor(...), so it carries a single rounding, and a rounded position that
// lands on an integer above the exact one is moved back to the cell below.  (With a
// rounded product the fraction is off by up to half an ulp of c*size, about 1e-5 texel at
// size 192, and the wrong cell extrapolates across a texel discontinuity.)  A position clamped to [-1, size] (including NaN) gets
// fraction 0: both neighbours are then the same edge texel.
__device__ __forceinline__ Axis coord_axis(float c, int size) {
  const float s = (float)size;
  const float q0 = fmaf(c, s, -0.5f);
  const float qc = fminf(fmaxf(q0, -1.0f), s);
  const float qf = floorf(qc);
  float f = fmaf(c, s, -0.5f - qf);
  int i = (int)qf;
  // the rounded position can land on the integer just above the exact one (never below):
  // then the exact fraction is negative and the cell is the one below
  if (f < 0.0f) {
    f += 1.0f;
    i -= 1;
  }
  f = (q0 == qc) ? f : 0.0f;
  Axis a;
  a.i0 = min(max(i, 0), size - 1);
  a.i1 = min(max(i + 1, 0), size - 1);
  a.w0 = 1.0f - f;
  a.w1 = f;
  return a;
}

// Axis on a grid of G nodes for the centre of texel x of a map S texels wide: position
// (x + 0.5) * G / S - 0.5 = ((2x + 1) G - S) / (2S), split into floor and fraction with
// integer arithmetic (exact); the common S = 4G case needs only shifts.
template <bool R4>
__device__ __forceinline__ Axis texel_axis(int x, int G, int S) {
  int q, r, den;
  if constexpr (R4) {
    const int num = 2 * x - 3;              // position * 8
    q = num >> 3;                           // floor division (arithmetic shift)
    r = num & 7;
    den = 8;
  } else {
    const int num = (2 * x + 1) * G - S;
    den = 2 * S;
    q = num >= 0 ? num / den : -((den - 1 - num) / den);
    r = num - q * den;
  }
  Axis a;
  a.i0 = min(max(q, 0), G - 1);
  a.i1 = min(max(q + 1, 0), G - 1);
  a.w1 = (float)r / (float)den;
  a.w0 = 1.0f - a.w1;
  return a;
}

struct Keys { int k0, k1; float w0, w1; };

// Periodic time keys t_k = k/T: t wraps into [0, 1); key T-1 blends into key 0.  The blend
// weight is one fused multiply-add of the exact product (t*T - k), a single rounding.
__device__ __forceinline__ Keys make_keys(float t, int T) {
  float tw = t - floorf(t);
  tw = (tw >= 0.0f && tw <= 1.0f) ? tw : 0.0f;   // non-finite t: any key (output is NaN)
  const float s = (float)T;
  const float kf = floorf(fmaf(tw, s, 0.0f));
  Keys k;
  k.w1 = fmaf(tw, s, -kf);
  int k0 = (int)kf;
  if (k.w1 < 0.0f) {            // rounded t*T landed on the key above the exact value
    k.w1 += 1.0f;
    k0 -= 1;
  }
  k.w0 = 1.0f - k.w1;
  k0 = k0 < 0 ? k0 + T : (k0 >= T ? k0 - T : k0);
  k.k0 = k0;
  k.k1 = k0 + 1 >= T ? 0 : k0 + 1;
  return k;
}

// Grid channels (2p, 2p+1) of node `node` ([T][Gh][Gw] flattened), 8 channels per node.
template <int GDT>
__device__ __forceinline__ float2 grid_pair(const void* grid, size_t node, int p) {
  if constexpr (GDT == NDGI_DTYPE_F16) {
    const uint32_t w = ((const uint32_t*)grid)[node * 4 + p];
    const _Float16 lo = __builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
    const _Float16 hi = __builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
    return make_float2((float)lo, (float)hi);
  }
  return ((const float2*)grid)[node * 4 + p];
}

// Grid sample of channels 2g, 2g+1: bilinear in space on the node axes, linear in time.
template <int GDT>
__device__ __forceinline__ float2 grid_sample(const ndgi_model& m, const Axis& ax, const Axis& ay, const Keys& k,
                                              int g) {
  float a = 0.0f, b = 0.0f;
#pragma unroll
  for (int tk = 0; tk < 2; ++tk) {
    const int key = tk ? k.k1 : k.k0;
    const float wt = tk ? k.w1 : k.w0;
#pragma unroll
    for (int yy = 0; yy < 2; ++yy) {
      const int gy = yy ? ay.i1 : ay.i0;
      const float wy = wt * (yy ? ay.w1 : ay.w0);
      const size_t row = ((size_t)key * m.Gh + gy) * m.Gw;
#pragma unroll
      for (int xx = 0; xx < 2; ++xx) {
        const int gx = xx ? ax.i1 : ax.i0;
        const float w = wy * (xx ? ax.w1 : ax.w0);
        const float2 v = grid_pair<GDT>(m.grid, row + gx, g);
        a = fmaf(w, v.x, a);
        b = fmaf(w, v.y, b);
      }
    }
  }
  return make_float2(a, b);
}

// Spatial channels 2g, 2g+1 of texel (x, y) as integers 0..255.
__device__ __forceinline__ uint2 spatial_pair(const ndgi_model& m, int x, int y, int g) {
  const uint4 b = *(const uint4*)(m.bc4 + ((size_t)(y >> 2) * (m.W >> 2) + (x >> 2)) * 64 + 16 * g);
  const uint32_t slot = 4u * (uint32_t)(y & 3) + (uint32_t)(x & 3);
  return make_uint2(bc4_texel(b.x, b.y, slot), bc4_texel(b.z, b.w, slot));
}

// ------------------------------------------------------- explicit-query features
// The decode of explicit (u, v, t) queries runs in two phases per wave pass of 64
// queries.  Phase A: lane l computes all 16 decoder inputs of query l in FP32 (x[0..7]
// spatial, x[8..15] grid) and writes them to a wave-private LDS block.  Phase B: the MFMA
// decoder reads them back in its operand layout (lane (g, j) of group q takes inputs
// 2g, 2g+1 and 8+2g, 8+2g+1 of query 16q + j).  Address and weight arithmetic is thus done
// once per query instead of once per lane group.  Every explicit-query decode uses these
// helpers, with the bilinear taps summed in the order (y0,x0), (y0,x1), (y1,x0), (y1,x1)
// and the keys k0 then k1, so that they agree bit for bit.

constexpr int kFeatStride = 20;   // floats per query row of the LDS block (80 B: 16-B aligned)

// Bilinear weights of the four taps, in summation order.
__device__ __forceinline__ void tap_weights(const Axis& ax, const Axis& ay, float w[4]) {
  w[0] = ay.w0 * ax.w0;
  w[1] = ay.w0 * ax.w1;
  w[2] = ay.w1 * ax.w0;
  w[3] = ay.w1 * ax.w1;
}

// Accumulate one grid node (8 channels) with weight w: FP16 nodes are 16 bytes (one uint4),
// FP32 nodes 32 bytes (two uint4).
template <int GDT>
__device__ __forceinline__ void grid_node_fma(const uint4* node, float w, float x[8]) {
  if constexpr (GDT == NDGI_DTYPE_F16) {
    const uint4 r = node[0];
    const uint32_t wd[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      x[2 * c] = fmaf(w, (float)__builtin_bit_cast(_Float16, (uint16_t)(wd[c] & 0xffffu)), x[2 * c]);
      x[2 * c + 1] = fmaf(w, (float)__builtin_bit_cast(_Float16, (uint16_t)(wd[c] >> 16)), x[2 * c + 1]);
    }
  } else {
    const uint4 a = node[0], b = node[1];
    const float vv[8] = {__uint_as_float(a.x), __uint_as_float(a.y), __uint_as_float(a.z), __uint_as_float(a.w),
                         __uint_as_float(b.x), __uint_as_float(b.y), __uint_as_float(b.z), __uint_as_float(b.w)};
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = fmaf(w, vv[c], x[c]);
  }
}

// Eight grid channels of query (u, v, t): bilinear on the node axes, linear in time.
// `node(key, gy, gx)` returns the address of a node (in HBM, or in a window staged in
// LDS); the weights and the summation order do not depend on where the nodes live.
template <int GDT, typename NodeAt>
__device__ __forceinline__ void query_grid8_at(const ndgi_model& m, float u, float v, float t, NodeAt node,
                                               float x[8]) {
  const Keys k = make_keys(t, m.T);
  const Axis gx = coord_axis(u, m.Gw), gy = coord_axis(v, m.Gh);
  float w[4];
  tap_weights(gx, gy, w);
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = 0.0f;
#pragma unroll
  for (int tk = 0; tk < 2; ++tk) {
    const int key = tk ? k.k1 : k.k0;
    const float wt = tk ? k.w1 : k.w0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      grid_node_fma<GDT>(node(key, (i & 2) ? gy.i1 : gy.i0, (i & 1) ? gx.i1 : gx.i0), wt * w[i], x);
  }
}

// The same with the nodes read from HBM.  Offsets are 32-bit (the host limits grids to
// 4 GiB).
template <int GDT>
__device__ __forceinline__ void query_grid8(const ndgi_model& m, float u, float v, float t, float x[8]) {
  const uint32_t plane = (uint32_t)m.Gh * (uint32_t)m.Gw;
  constexpr uint32_t kNodeBytes = GDT == NDGI_DTYPE_F16 ? 16u : 32u;
  const uint8_t* grid = (const uint8_t*)m.grid;
  query_grid8_at<GDT>(m, u, v, t, [&](int key, int gy, int gx) {
    return (const uint4*)(grid + ((uint32_t)key * plane + (uint32_t)gy * (uint32_t)m.Gw + (uint32_t)gx) * kNodeBytes);
  }, x);
}

// Eight spatial channels of a query, the four texels decoded straight from their BC4
// blocks (64 B per footprint: channel c in bytes 8c..8c+7).
__device__ __forceinline__ void spatial8_global(const ndgi_model& m, const Axis& ax, const Axis& ay, float x[8]) {
  float w[4];
  tap_weights(ax, ay, w);
  const uint32_t bw = (uint32_t)m.W >> 2;
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t y = (uint32_t)((i & 2) ? ay.i1 : ay.i0), xx = (uint32_t)((i & 1) ? ax.i1 : ax.i0);
    const uint8_t* fp = m.bc4 + ((y >> 2) * bw + (xx >> 2)) * 64u;
    const uint32_t slot = 4u * (y & 3u) + (xx & 3u);
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const uint4 b = *(const uint4*)(fp + 16 * h);
      x[2 * h] = fmaf(w[i], bc4_texel_f(b.x, b.y, slot), x[2 * h]);
      x[2 * h + 1] = fmaf(w[i], bc4_texel_f(b.z, b.w, slot), x[2 * h + 1]);
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] *= (1.0f / 255.0f);
}

// Eight spatial channels of a query from a decoded region in LDS: R x R texels from
// (tx0, ty0), 8 bytes per texel (channel c in byte c), row-major.
__device__ __forceinline__ void spatial8_lds(const uint2* reg, int R, int tx0, int ty0, const Axis& ax,
                                             const Axis& ay, float x[8]) {
  float w[4];
  tap_weights(ax, ay, w);
  const int o00 = (ay.i0 - ty0) * R + (ax.i0 - tx0);
  const int dx = ax.i1 - ax.i0, dy = (ay.i1 - ay.i0) * R;
  const int tap[4] = {o00, o00 + dx, o00 + dy, o00 + dy + dx};
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = 0.0f;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint2 p = reg[tap[i]];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      x[c] = fmaf(w[i], (float)((p.x >> (8 * c)) & 0xffu), x[c]);
      x[4 + c] = fmaf(w[i], (float)((p.y >> (8 * c)) & 0xffu), x[4 + c]);
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] *= (1.0f / 255.0f);
}

// Phase A -> B handoff in registers.  Lane l holds chunk c = {S_2c, S_2c+1, G_2c, G_2c+1}
// of its own query in r[c].  Viewing the wave as 4 rows of 16 lanes, the handoff is a 4 x 4
// transpose of chunks across rows: two v_permlane32_swap (rows 0,1 <-> 2,3) and two
// v_permlane16_swap (rows 0 <-> 1, 2 <-> 3) per chunk element.  Afterwards lane (g, j)
// holds in r[q] chunk g of query 16q + j, i.e. the decoder's K share for group q.
__device__ __forceinline__ void swap32(float& a, float& b) {
  const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(p[0]);
  b = __uint_as_float(p[1]);
}
__device__ __forceinline__ void swap16(float& a, float& b) {
  const auto p = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
  a = __uint_as_float(p[0]);
  b = __uint_as_float(p[1]);
}
// The transpose itself: r[c] of lane (row g, j) goes to r[g] of lane (row c, j).
__device__ __forceinline__ void transpose_rows(float r[4][4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    swap32(r[0][e], r[2][e]);   // rows 2,3 of r[0] <-> rows 0,1 of r[2]
    swap32(r[1][e], r[3][e]);
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    swap16(r[0][e], r[1][e]);   // odd rows of r[0] <-> even rows of r[1]
    swap16(r[2][e], r[3][e]);
  }
}
__device__ __forceinline__ void transpose_chunks(const float sp[8], const float gr[8], float r[4][4]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    r[c][0] = sp[2 * c];
    r[c][1] = sp[2 * c + 1];
    r[c][2] = gr[2 * c];
    r[c][3] = gr[2 * c + 1];
  }
  transpose_rows(r);
}

// Phase A store: this lane's 16 inputs into its row of the wave's block.
__device__ __forceinline__ void store_feats(float* feat, int lane, const float s[8], const float gr[8]) {
  float4* r = (float4*)(feat + lane * kFeatStride);
  r[0] = make_float4(s[0], s[1], s[2], s[3]);
  r[1] = make_float4(s[4], s[5], s[6], s[7]);
  r[2] = make_float4(gr[0], gr[1], gr[2], gr[3]);
  r[3] = make_float4(gr[4], gr[5], gr[6], gr[7]);
}

// Lane inputs at the centre of texel (x, y) (page / frame decode): the spatial sample is
// the texel itself; the grid axes come from texel_axis.
template <int GDT, bool R4>
__device__ __forceinline__ void texel_inputs(const ndgi_model& m, int x, int y, const Keys& k, int g, float f[4]) {
  const uint2 s = spatial_pair(m, x, y, g);
  const float2 gv = grid_sample<GDT>(m, texel_axis<R4>(x, m.Gw, m.W), texel_axis<R4>(y, m.Gh, m.H), k, g);
  f[0] = (float)s.x * (1.0f / 255.0f);
  f[1] = (float)s.y * (1.0f / 255.0f);
  f[2] = gv.x;
  f[3] = gv.y;
}

// ------------------------------------------------------------------ FP16 MFMA decoder
// Every FP16 operand that is not stored data (decoder inputs, hidden activations) is fed
// as a compensated pair v = hi + lo with lo = fp16(v - hi), so the products see about 22
// bits of v; the weights are exact in FP16.  The lo halves double the K depth of each
// layer: layer 1 (K = 16 -> 32) still takes one v_mfma_f32_16x16x32_f16 per 16 rows,
// layers 2 and 3 take two.  Without the lo terms the FP16 rounding of inputs and
// activations alone reaches 2.5e-3 relative output error on He-normal decoders.
//
// Two layer-1 input forms share the rest of the decoder:
//  * general (explicit queries): K slots [S_2g, S_2g+1, G_2g, G_2g+1] as hi, then as lo;
//  * texel centres: the spatial texel is an exact integer, fed as the FP16 value
//    1024 + u8 (bit pattern 0x6400 | u8) in both halves of K, against the hi and the lo
//    part of W1/255; the 1024 offset is removed through the bias.  Only the grid inputs
//    need a hi/lo split.

// d.lo16 = fp16(v0 - hi.lo16), d.hi16 = fp16(v1 - hi.hi16): the residuals of a packed
// pair of FP16 values against the FP32 values they came from (one v_fma_mix each).
__device__ __forceinline__ uint32_t resid_pair(uint32_t hi, float v0, float v1) {
  uint32_t d;
  // one statement writes both halves, so the result needs no initial value
  asm("v_fma_mixlo_f16 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]\n\t"
      "v_fma_mixhi_f16 %0, -%1, 1.0, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
      : "=&v"(d)
      : "v"(hi), "v"(v0), "v"(v1));
  return d;
}
// Same with the result clamped to [0, 1] (the hardware clamp bit).
__device__ __forceinline__ uint32_t resid_pair_clamp(uint32_t hi, float v0, float v1) {
  uint32_t d;
  asm("v_fma_mixlo_f16 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0] clamp\n\t"
      "v_fma_mixhi_f16 %0, -%1, 1.0, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0] clamp"
      : "=&v"(d)
      : "v"(hi), "v"(v0), "v"(v1));
  return d;
}

typedef _Float16 h2v __attribute__((ext_vector_type(2)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

// ReLU and hi/lo split of two 4-row output tiles into two 8-element K shares.  hi is
// rounded toward zero, so for a positive value the residual lies in [0, 1) and for a
// non-positive value it is <= 0: clamping the residual to [0, 1] is then exactly the ReLU
// of the lo part, and max(hi, 0) the ReLU of the hi part.
__device__ __forceinline__ void relu_split(const f4v& p0, const f4v& p1, h8v& hi, h8v& lo) {
  u4v H, Lo;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const f4v& p = t ? p1 : p0;
#pragma unroll
    for (int r = 0; r < 4; r += 2) {
      h2v v = __builtin_bit_cast(h2v, __builtin_amdgcn_cvt_pkrtz(p[r], p[r + 1]));
      v = __builtin_elementwise_max(v, (h2v){0, 0});
      const uint32_t hb = __builtin_bit_cast(uint32_t, v);
      H[2 * t + r / 2] = hb;
      Lo[2 * t + r / 2] = resid_pair_clamp(hb, p[r], p[r + 1]);
    }
  }
  hi = __builtin_bit_cast(h8v, H);
  lo = __builtin_bit_cast(h8v, Lo);
}

// hi/lo split of four general inputs into the layer-1 K share [hi(4), lo(4)].
__device__ __forceinline__ h8v split_inputs(const float f[4]) {
  const uint32_t h01 = __builtin_bit_cast(uint32_t, (h2v){(_Float16)f[0], (_Float16)f[1]});
  const uint32_t h23 = __builtin_bit_cast(uint32_t, (h2v){(_Float16)f[2], (_Float16)f[3]});
  const u4v x = {h01, h23, resid_pair(h01, f[0], f[1]), resid_pair(h23, f[2], f[3])};
  return __builtin_bit_cast(h8v, x);
}

// Layer-1 K share at a texel centre: spatial pair given as 0x6400|u8 halves, grid pair split.
__device__ __forceinline__ h8v texel_x(uint32_t sp, float ga, float gb) {
  const uint32_t gh = __builtin_bit_cast(uint32_t, (h2v){(_Float16)ga, (_Float16)gb});
  const u4v x = {sp, gh, sp, resid_pair(gh, ga, gb)};
  return __builtin_bit_cast(h8v, x);
}

struct Dec16 {
  h8v a1[2];   // layer 1, rows 16mc + i (see load_dec16 for the K slots)
  h8v a2[2];   // W2 rows 16mo + i, units unit_of(g, 0..7)
  h8v a3[4];   // W3 placed at rows 4q..4q+2 for group q, zero elsewhere
  f4v c1[2], c2[2], c3;   // biases in C layout (rows 4g..4g+3)
};

// TEXEL = false: layer-1 slots e = 0..3 take W1 at input_of(g, e), slots 4..7 the same
// weights (they multiply the lo halves).  TEXEL = true: slots 0, 1 take hi(W1/255) of
// spatial 2g, 2g+1, slots 4, 5 lo(W1/255), slots 2, 3 and 6, 7 the grid weights; c1 has
// 1024 * sum_s (hi + lo) removed.
template <int MDT, bool TEXEL>
__device__ __forceinline__ void load_dec16(Dec16& d, const void* mlp, int lane) {
  const int g = lane >> 4, i = lane & 15;
#pragma unroll
  for (int mc = 0; mc < 2; ++mc) {
    const int u = 16 * mc + i;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int in = input_of(g, e & 3);
      const float w = ld<MDT>(mlp, kOffW1 + u * 16 + in);
      if (TEXEL && (e & 3) < 2) {
        const float ws = w * (1.0f / 255.0f);
        const _Float16 hi = (_Float16)ws;
        d.a1[mc][e] = e < 4 ? hi : (_Float16)(ws - (float)hi);
      } else {
        d.a1[mc][e] = (_Float16)w;
      }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e)
      d.a2[mc][e] = (_Float16)ld<MDT>(mlp, kOffW2 + u * 32 + unit_of(g, e));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ur = 16 * mc + 4 * g + r;
      float b = ld<MDT>(mlp, kOffB1 + ur);
      if (TEXEL) {
        float off = 0.0f;
#pragma unroll
        for (int sc = 0; sc < 8; ++sc) {
          const float ws = ld<MDT>(mlp, kOffW1 + ur * 16 + sc) * (1.0f / 255.0f);
          const _Float16 hi = (_Float16)ws;
          off += (float)hi + (float)(_Float16)(ws - (float)hi);
        }
        b -= 1024.0f * off;
      }
      d.c1[mc][r] = b;
      d.c2[mc][r] = ld<MDT>(mlp, kOffB2 + ur);
    }
  }
  // every load is unconditional (clamped index, then a select): a conditional load would
  // be branched around and serialise the whole set
  float w3[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) w3[e] = ld<MDT>(mlp, kOffW3 + min(i & 3, 2) * 32 + unit_of(g, e));
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int e = 0; e < 8; ++e) d.a3[q][e] = ((i >> 2) == q && (i & 3) < 3) ? (_Float16)w3[e] : (_Float16)0.0f;
#pragma unroll
  for (int r = 0; r < 4; ++r) d.c3[r] = r < 3 ? ld<MDT>(mlp, kOffB3 + r) : 0.0f;
}

// One 16-texel group through the decoder from its layer-1 K share; the output layer
// accumulates into acc.
__device__ __forceinline__ void dec16_group(const Dec16& d, const h8v& x, int q, f4v& acc) {
  const f4v p0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(d.a1[0], x, d.c1[0], 0, 0, 0);
  const f4v p1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(d.a1[1], x, d.c1[1], 0, 0, 0);
  h8v h, hl;
  relu_split(p0, p1, h, hl);
  f4v r0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(d.a2[0], h, d.c2[0], 0, 0, 0);
  f4v r1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(d.a2[1], h, d.c2[1], 0, 0, 0);
  r0 = __builtin_amdgcn_mfma_f32_16x16x32_f16(d.a2[0], hl, r0, 0, 0, 0);
  r1 = __builtin_amdgcn_mfma_f32_16x16x32_f16(d.a2[1], hl, r1, 0, 0, 0);
  h8v h2, h2l;
  relu_split(r0, r1, h2, h2l);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(d.a3[q], h2, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(d.a3[q], h2l, acc, 0, 0, 0);
}

// ------------------------------------------------------------------ FP32 MFMA decoder
// v_mfma_f32_16x16x4_f32: lane (g, i) supplies one K element (k = g); layer K depths 16
// and 32 are covered by 4 and 8 chained MFMAs, step m taking element m of the lane's
// share (input_of(g, m) in layer 1, unit_of(g, m) in layers 2-3).
struct Dec32 {
  float a1[2][4];
  float a2[2][8];
  float a3[4][8];
  f4v c1[2], c2[2], c3;
};

template <int MDT>
__device__ __forceinline__ void load_dec32(Dec32& d, const void* mlp, int lane) {
  const int g = lane >> 4, i = lane & 15;
#pragma unroll
  for (int mc = 0; mc < 2; ++mc) {
#pragma unroll
    for (int e = 0; e < 4; ++e) d.a1[mc][e] = ld<MDT>(mlp, kOffW1 + (16 * mc + i) * 16 + input_of(g, e));
#pragma unroll
    for (int e = 0; e < 8; ++e) d.a2[mc][e] = ld<MDT>(mlp, kOffW2 + (16 * mc + i) * 32 + unit_of(g, e));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      d.c1[mc][r] = ld<MDT>(mlp, kOffB1 + 16 * mc + 4 * g + r);
      d.c2[mc][r] = ld<MDT>(mlp, kOffB2 + 16 * mc + 4 * g + r);
    }
  }
  float w3[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) w3[e] = ld<MDT>(mlp, kOffW3 + min(i & 3, 2) * 32 + unit_of(g, e));
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int e = 0; e < 8; ++e) d.a3[q][e] = ((i >> 2) == q && (i & 3) < 3) ? w3[e] : 0.0f;
#pragma unroll
  for (int r = 0; r < 4; ++r) d.c3[r] = r < 3 ? ld<MDT>(mlp, kOffB3 + r) : 0.0f;
}

__device__ __forceinline__ void dec32_group(const Dec32& d, const float f[4], int q, f4v& acc) {
  f4v p0 = d.c1[0], p1 = d.c1[1];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    p0 = __builtin_amdgcn_mfma_f32_16x16x4f32(d.a1[0][m], f[m], p0, 0, 0, 0);
    p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(d.a1[1][m], f[m], p1, 0, 0, 0);
  }
  float h[8];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    h[r] = fmaxf(p0[r], 0.0f);
    h[4 + r] = fmaxf(p1[r], 0.0f);
  }
  f4v r0 = d.c2[0], r1 = d.c2[1];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    r0 = __builtin_amdgcn_mfma_f32_16x16x4f32(d.a2[0][m], h[m], r0, 0, 0, 0);
    r1 = __builtin_amdgcn_mfma_f32_16x16x4f32(d.a2[1][m], h[m], r1, 0, 0, 0);
  }
  float h2[8];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    h2[r] = fmaxf(r0[r], 0.0f);
    h2[4 + r] = fmaxf(r1[r], 0.0f);
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(d.a3[q][m], h2[m], acc, 0, 0, 0);
}

// Generic wrappers selected by precision.
template <int PREC> struct Dec;
template <> struct Dec<NDGI_PREC_F16> {
  Dec16 d;
  __device__ __forceinline__ void load(const void* mlp, int dt, int lane) {
    if (dt == NDGI_DTYPE_F16) load_dec16<NDGI_DTYPE_F16, false>(d, mlp, lane);
    else load_dec16<NDGI_DTYPE_F32, false>(d, mlp, lane);
  }
  __device__ __forceinline__ void group(const float f[4], int q, f4v& acc) const {
    dec16_group(d, split_inputs(f), q, acc);
  }
  __device__ __forceinline__ f4v bias3() const { return d.c3; }
};
template <> struct Dec<NDGI_PREC_F32> {
  Dec32 d;
  __device__ __forceinline__ void load(const void* mlp, int dt, int lane) {
    if (dt == NDGI_DTYPE_F16) load_dec32<NDGI_DTYPE_F16>(d, mlp, lane);
    else load_dec32<NDGI_DTYPE_F32>(d, mlp, lane);
  }
  __device__ __forceinline__ void group(const float f[4], int q, f4v& acc) const { dec32_group(d, f, q, acc); }
  __device__ __forceinline__ f4v bias3() const { return d.c3; }
};

// Phase B from registers: the decoder over the wave's 64 queries after the handoff; lane l
// ends with the output-layer values of query l.
template <int PREC>
__device__ __forceinline__ f4v decode_regs(const Dec<PREC>& dec, const float sp[8], const float gr[8]) {
  float r[4][4];
  transpose_chunks(sp, gr, r);
  f4v acc = dec.bias3();
#pragma unroll
  for (int q = 0; q < 4; ++q) dec.group(r[q], q, acc);
  return acc;
}

// Phase B: the decoder over the 64 queries of a wave's feature block; lane l ends with
// the output-layer values of query l.
template <int PREC>
__device__ __forceinline__ f4v decode_feats(const Dec<PREC>& dec, const float* feat, int g, int j) {
  f4v acc = dec.bias3();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float* r = feat + (16 * q + j) * kFeatStride;
    const float2 sp = *(const float2*)(r + 2 * g);
    const float2 gr = *(const float2*)(r + 8 + 2 * g);
    const float f[4] = {sp.x, sp.y, gr.x, gr.y};
    dec.group(f, q, acc);
  }
  return acc;
}

// Store the RGB of one texel: exp of the output layer, FP16 (rounded once) or FP32.
template <int PREC>
__device__ __forceinline__ void store_rgb(void* out, size_t idx, const f4v& z, bool nan_out) {
  if constexpr (PREC == NDGI_PREC_F16) {
    float r = __expf(z[0]), g = __expf(z[1]), b = __expf(z[2]);
    if (nan_out) r = g = b = __builtin_nanf("");
    _Float16* o = (_Float16*)out + idx * 3;
    o[0] = (_Float16)r;
    o[1] = (_Float16)g;
    o[2] = (_Float16)b;
  } else {
    float r = expf(z[0]), g = expf(z[1]), b = expf(z[2]);
    if (nan_out) r = g = b = __builtin_nanf("");
    float* o = (float*)out + idx * 3;
    o[0] = r;
    o[1] = g;
    o[2] = b;
  }
}

}  // namespace ndgi
