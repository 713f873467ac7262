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

__device__ __forceinline__ float mlp_at(const void* p, int dt, int i) {
  return dt == NDGI_DTYPE_F16 ? (float)((const _Float16*)p)[i] : ((const float*)p)[i];
}

// Decoder input fed by element e (0..3) of lane group g in the first layer:
// spatial 2g, 2g+1, grid 2g, 2g+1 (inputs are ordered [S0..S7, G0..G7]).
__device__ __forceinline__ int input_of(int g, int e) { return e < 2 ? 2 * g + e : 8 + 2 * g + (e - 2); }
// Hidden unit fed by element e (0..7) of lane group g in a 32-deep K operand: the
// lane's rows 4g..4g+3 of the first and of the second 16-row output tile.
__device__ __forceinline__ int unit_of(int g, int e) { return e < 4 ? 4 * g + e : 16 + 4 * g + (e - 4); }

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

// ------------------------------------------------------------------ sampling helpers
struct Axis { int i0, i1; float w0, w1; };

// Axis of normalised coordinate c with the texel-centre convention: continuous position
// c*size - 0.5, neighbours floor() and floor()+1 clamped to [0, size-1].  The fraction is
// one fused multiply-add of the exact product, c*size - 0.5 - floor(...), so it carries a
// single rounding (a separately rounded product would add up to half an ulp of c*size,
// about 1e-5 texel at size 192).  A position clamped to [-1, size] (including NaN) gets
// fraction 0: both neighbours are then the same edge texel.
__device__ __forceinline__ Axis coord_axis(float c, int size) {
  const float s = (float)size;
  const float q0 = fmaf(c, s, -0.5f);
  const float qc = fminf(fmaxf(q0, -1.0f), s);
  const float qf = floorf(qc);
  float f = fmaf(c, s, -0.5f - qf);
  f = (q0 == qc) ? f : 0.0f;
  const int i = (int)qf;
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
__device__ __forceinline__ Axis texel_axis(int x, int G, int S) {
  int q, r, den;
  if (S == 4 * G) {
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
  k.w0 = 1.0f - k.w1;
  int k0 = (int)kf;
  k0 = k0 >= T ? k0 - T : k0;
  k.k0 = k0;
  k.k1 = k0 + 1 >= T ? 0 : k0 + 1;
  return k;
}

// Grid channels (2p, 2p+1) of node `node` ([T][Gh][Gw] flattened), 8 channels per node.
__device__ __forceinline__ float2 grid_pair(const void* grid, int dt, size_t node, int p) {
  if (dt == NDGI_DTYPE_F16) {
    const uint32_t w = ((const uint32_t*)grid)[node * 4 + p];
    const _Float16 lo = __builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu));
    const _Float16 hi = __builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
    return make_float2((float)lo, (float)hi);
  }
  return ((const float2*)grid)[node * 4 + p];
}

// Grid sample of channels 2g, 2g+1: bilinear in space on the node axes, linear in time.
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
        const float2 v = grid_pair(m.grid, m.grid_dtype, row + gx, g);
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

// Lane inputs for an explicit query (u, v, t).
__device__ __forceinline__ void query_inputs(const ndgi_model& m, float u, float v, float t, int g, float f[4]) {
  const Axis ax = coord_axis(u, m.W);
  const Axis ay = coord_axis(v, m.H);
  float s0 = 0.0f, s1 = 0.0f;
#pragma unroll
  for (int yy = 0; yy < 2; ++yy) {
    const int y = yy ? ay.i1 : ay.i0;
    const float wy = yy ? ay.w1 : ay.w0;
#pragma unroll
    for (int xx = 0; xx < 2; ++xx) {
      const int x = xx ? ax.i1 : ax.i0;
      const float w = wy * (xx ? ax.w1 : ax.w0);
      const uint2 s = spatial_pair(m, x, y, g);
      s0 = fmaf(w, (float)s.x, s0);
      s1 = fmaf(w, (float)s.y, s1);
    }
  }
  const Keys k = make_keys(t, m.T);
  const float2 gv = grid_sample(m, coord_axis(u, m.Gw), coord_axis(v, m.Gh), k, g);
  f[0] = s0 * (1.0f / 255.0f);
  f[1] = s1 * (1.0f / 255.0f);
  f[2] = gv.x;
  f[3] = gv.y;
}

// Lane inputs at the centre of texel (x, y) (page / frame decode): the spatial sample is
// the texel itself; the grid axes come from texel_axis.
__device__ __forceinline__ void texel_inputs(const ndgi_model& m, int x, int y, const Keys& k, int g, float f[4]) {
  const uint2 s = spatial_pair(m, x, y, g);
  const float2 gv = grid_sample(m, texel_axis(x, m.Gw, m.W), texel_axis(y, m.Gh, m.H), k, g);
  f[0] = (float)s.x * (1.0f / 255.0f);
  f[1] = (float)s.y * (1.0f / 255.0f);
  f[2] = gv.x;
  f[3] = gv.y;
}

// ------------------------------------------------------------------ FP16 MFMA decoder
// Every FP16 operand that is not stored data (decoder inputs, hidden activations) is fed
// as a compensated pair v = hi + lo, hi = fp16(v), lo = fp16(v - hi), so the products see
// about 22 bits of v; the weights are exact in FP16.  The lo halves double the K depth of
// each layer: layer 1 (K = 16 -> 32) still takes one v_mfma_f32_16x16x32_f16 per 16 rows,
// layers 2 and 3 take two.  Without the lo terms the FP16 rounding of inputs and
// activations alone reaches 2.5e-3 relative output error on He-normal decoders.
struct Dec16 {
  h8v a1[2];   // W1 rows 16mc + i: inputs input_of(g, 0..3), then the same four again (lo)
  h8v a2[2];   // W2 rows 16mo + i, units unit_of(g, 0..7)
  h8v a3[4];   // W3 placed at rows 4q..4q+2 for group q, zero elsewhere
  f4v c1[2], c2[2], c3;   // biases in C layout (rows 4g..4g+3)
};

__device__ __forceinline__ void load_dec16(Dec16& d, const void* mlp, int dt, int lane) {
  const int g = lane >> 4, i = lane & 15;
#pragma unroll
  for (int mc = 0; mc < 2; ++mc) {
#pragma unroll
    for (int e = 0; e < 8; ++e)
      d.a1[mc][e] = (_Float16)mlp_at(mlp, dt, kOffW1 + (16 * mc + i) * 16 + input_of(g, e & 3));
#pragma unroll
    for (int e = 0; e < 8; ++e)
      d.a2[mc][e] = (_Float16)mlp_at(mlp, dt, kOffW2 + (16 * mc + i) * 32 + unit_of(g, e));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      d.c1[mc][r] = mlp_at(mlp, dt, kOffB1 + 16 * mc + 4 * g + r);
      d.c2[mc][r] = mlp_at(mlp, dt, kOffB2 + 16 * mc + 4 * g + r);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int e = 0; e < 8; ++e)
      d.a3[q][e] = ((i >> 2) == q && (i & 3) < 3)
                       ? (_Float16)mlp_at(mlp, dt, kOffW3 + (i & 3) * 32 + unit_of(g, e))
                       : (_Float16)0.0f;
#pragma unroll
  for (int r = 0; r < 4; ++r) d.c3[r] = r < 3 ? mlp_at(mlp, dt, kOffB3 + r) : 0.0f;
}

// hi/lo split of ReLU'd pre-activations (two 4-row tiles) into two 8-element K shares
__device__ __forceinline__ void relu_split(const f4v& p0, const f4v& p1, h8v& hi, h8v& lo) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float a = __builtin_fmaxf(p0[r], 0.0f), b = __builtin_fmaxf(p1[r], 0.0f);
    hi[r] = (_Float16)a;
    hi[4 + r] = (_Float16)b;
    lo[r] = (_Float16)(a - (float)hi[r]);
    lo[4 + r] = (_Float16)(b - (float)hi[4 + r]);
  }
}

// One 16-texel group through the decoder; the output layer accumulates into acc.
__device__ __forceinline__ void dec16_group(const Dec16& d, const float f[4], int q, f4v& acc) {
  h8v x;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    x[e] = (_Float16)f[e];
    x[4 + e] = (_Float16)(f[e] - (float)x[e]);
  }
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

__device__ __forceinline__ void load_dec32(Dec32& d, const void* mlp, int dt, int lane) {
  const int g = lane >> 4, i = lane & 15;
#pragma unroll
  for (int mc = 0; mc < 2; ++mc) {
#pragma unroll
    for (int e = 0; e < 4; ++e) d.a1[mc][e] = mlp_at(mlp, dt, kOffW1 + (16 * mc + i) * 16 + input_of(g, e));
#pragma unroll
    for (int e = 0; e < 8; ++e) d.a2[mc][e] = mlp_at(mlp, dt, kOffW2 + (16 * mc + i) * 32 + unit_of(g, e));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      d.c1[mc][r] = mlp_at(mlp, dt, kOffB1 + 16 * mc + 4 * g + r);
      d.c2[mc][r] = mlp_at(mlp, dt, kOffB2 + 16 * mc + 4 * g + r);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int e = 0; e < 8; ++e)
      d.a3[q][e] = ((i >> 2) == q && (i & 3) < 3) ? mlp_at(mlp, dt, kOffW3 + (i & 3) * 32 + unit_of(g, e)) : 0.0f;
#pragma unroll
  for (int r = 0; r < 4; ++r) d.c3[r] = r < 3 ? mlp_at(mlp, dt, kOffB3 + r) : 0.0f;
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
  __device__ __forceinline__ void load(const void* mlp, int dt, int lane) { load_dec16(d, mlp, dt, lane); }
  __device__ __forceinline__ void group(const float f[4], int q, f4v& acc) const { dec16_group(d, f, q, acc); }
  __device__ __forceinline__ f4v bias3() const { return d.c3; }
};
template <> struct Dec<NDGI_PREC_F32> {
  Dec32 d;
  __device__ __forceinline__ void load(const void* mlp, int dt, int lane) { load_dec32(d, mlp, dt, lane); }
  __device__ __forceinline__ void group(const float f[4], int q, f4v& acc) const { dec32_group(d, f, q, acc); }
  __device__ __forceinline__ f4v bias3() const { return d.c3; }
};

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
