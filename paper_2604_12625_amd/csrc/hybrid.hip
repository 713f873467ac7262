// Decode of the paper's hybrid layout (Sec. 3.3, Eq. 4-5): F_uvt (4 channels in time
// slices, each slice block-compressed), F_uv (4 channels, block-compressed: BC4 per channel
// or BC7 blocks of modes 4-6), F_ut and F_vt (2 channels each, 8-bit)
// and gamma(t) feed a 16 -> h -> h -> 3 decoder with GELU hidden layers and a linear
// output (Sec. 4), h = 16 or 64.
//
// Decoder on MFMA.  A wave decodes 64 texels per pass as 4 groups of 16.  After the
// register handoff lane (g, j) holds decoder inputs 4g..4g+3 of texel 16q + j for group q
// (chunk 0 = V_uvt, 1 = V_uv, 2 = V_ut and V_vt, 3 = gamma).  Hidden units are MFMA rows in
// blocks of 16; the C layout of a block (lane holds rows 4g..4g+3 of column j) is the
// lane's K share of that block for the next layer, so no data moves between layers.
//  * FP16: one v_mfma_f32_16x16x32_f16 per (row block, K block).  K slots 0..3 of lane
//    group g carry the FP16 value ("hi") of units 4g..4g+3 of the K block and slots 4..7
//    their residual fp16(v - hi) ("lo"), so inputs and activations enter with about 22
//    bits while the weights (exact in FP16) appear in both halves.
//  * FP32: v_mfma_f32_16x16x4_f32, step r feeding unit 4g + r of the K block.
// The weights in that K order (the MFMA A operands) are laid out once per model in an LDS
// table of 16-byte lane entries: "chunk" = 64 lanes x 16 bytes (8 FP16 slots or 4 FP32
// steps); the output layer's chunk holds W3 on rows 4k..4k+2 of every row quad k, and group
// q keeps quad q only, so the 4 groups write rows 4q..4q+2 of one accumulator and after
// them lane l owns the RGB of texel l of the pass.
#include "hybrid.hpp"
#include "internal.hpp"

namespace ndgi {

template <int HD>
struct HybTab {
  u4v a[HybShape<HD>::kChunks * 64];
  float b1[HD], b2[HD];
  float b3[4];
};

// Build the decoder table of a model (all threads of the workgroup; the caller
// synchronises before use).
template <int PREC, int HD, int MDT>
__device__ void hyb_build_dt(HybTab<HD>& T, const void* mlp) {
  using S = HybShape<HD>;
  for (int idx = threadIdx.x; idx < S::kChunks * 64; idx += blockDim.x) {
    const int c = idx >> 6, lane = idx & 63, g = lane >> 4, i = lane & 15;
    int base, kbase;   // offset of the row in the packed vector (or -1 for a zero row), first unit
    if (c < S::kL2) {
      base = S::oW1 + (16 * c + i) * NDGI_HYBRID_IN;
      kbase = 4 * g;
    } else if (c < S::kL3) {
      const int ob = (c - S::kL2) / S::NB, kb = (c - S::kL2) % S::NB;
      base = S::oW2 + (16 * ob + i) * HD;
      kbase = 16 * kb + 4 * g;
    } else {
      // output row (i & 3) on every row quad; hyb_group keeps quad q for group q
      const int kb = c - S::kL3;
      base = (i & 3) < 3 ? S::oW3 + (i & 3) * HD : -1;
      kbase = 16 * kb + 4 * g;
    }
    // loads are unconditional (clamped row), the zero rows select afterwards
    const int row = base < 0 ? S::oW3 : base;
    float w[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) w[r] = base < 0 ? 0.0f : ld<MDT>(mlp, row + kbase + r);
    if constexpr (PREC == NDGI_PREC_F16) {
      h8v h;
#pragma unroll
      for (int e = 0; e < 8; ++e) h[e] = (_Float16)w[e & 3];
      T.a[idx] = __builtin_bit_cast(u4v, h);
    } else {
      T.a[idx] = (u4v){__float_as_uint(w[0]), __float_as_uint(w[1]), __float_as_uint(w[2]), __float_as_uint(w[3])};
    }
  }
  for (int j = threadIdx.x; j < HD; j += blockDim.x) {
    T.b1[j] = ld<MDT>(mlp, S::oB1 + j);
    T.b2[j] = ld<MDT>(mlp, S::oB2 + j);
  }
  if (threadIdx.x < 4) T.b3[threadIdx.x] = threadIdx.x < 3 ? ld<MDT>(mlp, S::oB3 + threadIdx.x) : 0.0f;
}

template <int PREC, int HD>
__device__ void hyb_build(HybTab<HD>& T, const void* mlp, int mlp_dtype) {
  if (mlp_dtype == NDGI_DTYPE_F16) hyb_build_dt<PREC, HD, NDGI_DTYPE_F16>(T, mlp);
  else hyb_build_dt<PREC, HD, NDGI_DTYPE_F32>(T, mlp);
}

// One group of 16 texels through the decoder; x = this lane's K share of layer 1 (inputs
// 4g..4g+3); the output layer accumulates into acc.
template <int PREC, int HD>
__device__ __forceinline__ void hyb_group(const HybTab<HD>& T, const float x[4], int q, int lane, f4v& acc) {
  using S = HybShape<HD>;
  constexpr int NB = S::NB;
  const int g = lane >> 4;
  const bool own = ((lane & 15) >> 2) == q;   // A rows 4q..4q+2 carry the output layer of group q
  if constexpr (PREC == NDGI_PREC_F16) {
    auto A = [&](int c) { return __builtin_bit_cast(h8v, T.a[c * 64 + lane]); };
    const h8v X = split_inputs(x);
    h8v H1[NB], H2[NB];
#pragma unroll
    for (int mb = 0; mb < NB; ++mb) {
      const f4v p = __builtin_amdgcn_mfma_f32_16x16x32_f16(A(S::kL1 + mb), X, *(const f4v*)&T.b1[16 * mb + 4 * g],
                                                           0, 0, 0);
      const float h[4] = {gelu<PREC>(p[0]), gelu<PREC>(p[1]), gelu<PREC>(p[2]), gelu<PREC>(p[3])};
      H1[mb] = split_inputs(h);
    }
#pragma unroll
    for (int ob = 0; ob < NB; ++ob) {
      f4v a = *(const f4v*)&T.b2[16 * ob + 4 * g];
#pragma unroll
      for (int kb = 0; kb < NB; ++kb) a = __builtin_amdgcn_mfma_f32_16x16x32_f16(A(S::kL2 + ob * NB + kb), H1[kb], a, 0, 0, 0);
      const float h[4] = {gelu<PREC>(a[0]), gelu<PREC>(a[1]), gelu<PREC>(a[2]), gelu<PREC>(a[3])};
      H2[ob] = split_inputs(h);
    }
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
      const h8v a3 = own ? A(S::kL3 + kb) : (h8v){0, 0, 0, 0, 0, 0, 0, 0};
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a3, H2[kb], acc, 0, 0, 0);
    }
  } else {
    auto A = [&](int c) { return __builtin_bit_cast(f4v, T.a[c * 64 + lane]); };
    float h1[NB][4], h2[NB][4];
#pragma unroll
    for (int mb = 0; mb < NB; ++mb) {
      const f4v w = A(S::kL1 + mb);
      f4v p = *(const f4v*)&T.b1[16 * mb + 4 * g];
#pragma unroll
      for (int r = 0; r < 4; ++r) p = __builtin_amdgcn_mfma_f32_16x16x4f32(w[r], x[r], p, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) h1[mb][r] = gelu<PREC>(p[r]);
    }
#pragma unroll
    for (int ob = 0; ob < NB; ++ob) {
      f4v a = *(const f4v*)&T.b2[16 * ob + 4 * g];
#pragma unroll
      for (int kb = 0; kb < NB; ++kb) {
        const f4v w = A(S::kL2 + ob * NB + kb);
#pragma unroll
        for (int r = 0; r < 4; ++r) a = __builtin_amdgcn_mfma_f32_16x16x4f32(w[r], h1[kb][r], a, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) h2[ob][r] = gelu<PREC>(a[r]);
    }
#pragma unroll
    for (int kb = 0; kb < NB; ++kb) {
      const f4v w = own ? A(S::kL3 + kb) : (f4v){0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w[r], h2[kb][r], acc, 0, 0, 0);
    }
  }
}

// The decoder over a wave's 64 texels: r[c] holds chunk c of this lane's own texel on
// entry; returns the output of the lane's texel.
template <int PREC, int HD>
__device__ __forceinline__ f4v hyb_decode(const HybTab<HD>& T, float r[4][4], int lane) {
  transpose_rows(r);
  f4v acc = *(const f4v*)T.b3;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    hyb_group<PREC, HD>(T, r[q], q, lane, acc);
    // groups are not interleaved: each one's activations are dead before the next starts
    __builtin_amdgcn_sched_barrier(0);
  }
  return acc;
}

// Linear output (no activation); NaN for queries with a non-finite coordinate.
template <int PREC>
__device__ __forceinline__ void store_lin(void* out, size_t idx, const f4v& z, bool nan_out) {
  float r = z[0], g = z[1], b = z[2];
  if (nan_out) r = g = b = __builtin_nanf("");
  if constexpr (PREC == NDGI_PREC_F16) {
    _Float16* o = (_Float16*)out + idx * 3;
    o[0] = (_Float16)r;
    o[1] = (_Float16)g;
    o[2] = (_Float16)b;
  } else {
    float* o = (float*)out + idx * 3;
    o[0] = r;
    o[1] = g;
    o[2] = b;
  }
}

// ---------------------------------------------------------------------- time axis
struct HybTime {
  NodeT s;      // F_uvt slices
  NodeT k;      // F_ut / F_vt rows
  float g[4];   // gamma(t)
};

template <typename KeyAt>
__device__ __forceinline__ HybTime hyb_time(const ndgi_hybrid_model& m, float t, KeyAt key) {
  const float tc = clamp01(t);
  const float tau = key_tau(tc, m.n_keys, key);
  HybTime h;
  h.s = node_axis(tau, m.S);
  h.k = node_axis(tau, m.Tt);
  float s, c;
  sincospif(tc, &s, &c);
  h.g[0] = s;
  h.g[1] = c;
  h.g[2] = 2.0f * s * c;
  h.g[3] = fmaf(c, c, -s * s);
  return h;
}

// ---------------------------------------------------------------------- feature maps
// Four channels of texel slot `slot` of a 32-byte BC4 footprint (channel c in bytes 8c..8c+7).
__device__ __forceinline__ void bc4_fp4(const uint8_t* fp, uint32_t slot, float v[4]) {
  const u4v a = ((const u4v*)fp)[0], b = ((const u4v*)fp)[1];
  v[0] = bc4_texel_f(a.x, a.y, slot);
  v[1] = bc4_texel_f(a.z, a.w, slot);
  v[2] = bc4_texel_f(b.x, b.y, slot);
  v[3] = bc4_texel_f(b.z, b.w, slot);
}

__device__ __forceinline__ void bc4_fp4_regs(const u4v& a, const u4v& b, uint32_t slot, float v[4]) {
  v[0] = bc4_texel_f(a.x, a.y, slot);
  v[1] = bc4_texel_f(a.z, a.w, slot);
  v[2] = bc4_texel_f(b.x, b.y, slot);
  v[3] = bc4_texel_f(b.z, b.w, slot);
}

// Bits [pos, pos + n) (n <= 8) of a BC7 block held as a 128-bit little-endian value.
__device__ __forceinline__ uint32_t bc7_bits(uint64_t lo, uint64_t hi, uint32_t pos, uint32_t n) {
  const uint64_t v = pos >= 64u ? hi >> (pos - 64u) : (pos == 0u ? lo : (lo >> pos) | (hi << (64u - pos)));
  return (uint32_t)v & ((1u << n) - 1u);
}
// Index of texel `slot` in an index set of b-bit indices starting at bit pos (texel 0 has
// b - 1 bits).
__device__ __forceinline__ uint32_t bc7_index(uint64_t lo, uint64_t hi, uint32_t pos, uint32_t b, uint32_t slot) {
  return slot ? bc7_bits(lo, hi, pos + b - 1u + b * (slot - 1u), b) : bc7_bits(lo, hi, pos, b - 1u);
}
// n-bit endpoint value as 8 bits: the top bits replicated below.
__device__ __forceinline__ uint32_t bc7_expand(uint32_t v, uint32_t n) { return (v << (8u - n)) | (v >> (2u * n - 8u)); }

// Four channels of texel `slot` of a BC7 block (b = the 16 bytes as a 128-bit little-endian
// value) in mode 4, 5 or 6, the single-subset modes with four channels; other modes give 0.
//  * mode 6 (bits 0..6 = 1000000b): 7-bit endpoint values R0 R1 G0 G1 B0 B1 A0 A1 at bits
//    7..62, p-bits at 63 and 64, one 4-bit index per texel from bit 65; endpoint (v << 1) | p;
//  * mode 5 (bits 0..5 = 100000b): rotation at 6..7, 7-bit colour endpoints R0 .. B1 from
//    bit 8, 8-bit alpha endpoints at 50 and 58, 2-bit colour indices from 66 and 2-bit
//    alpha indices from 97;
//  * mode 4 (bits 0..4 = 10000b): rotation at 5..6, index selection at 7, 5-bit colour
//    endpoints from bit 8, 6-bit alpha endpoints at 38 and 44, a 2-bit index set from 50 and
//    a 3-bit set from 81 (colour takes the 3-bit set when the selection bit is 1).
// An n-bit endpoint is (v << (8 - n)) | (v >> (2n - 8)); texel ((64 - w) E0 + w E1 + 32) >> 6
// with w = (64 J + (2^b - 1) / 2) / (2^b - 1), which equals the format's b-bit weight table;
// rotation r > 0 exchanges channel r - 1 with channel 3 after decoding.
__device__ __forceinline__ void bc7_fp4_regs(const u4v& b, uint32_t slot, float v[4]) {
  const uint64_t lo = ((uint64_t)b.y << 32) | b.x, hi = ((uint64_t)b.w << 32) | b.z;
  const uint32_t m = b.x & 0xffu;
  uint32_t e0[4], e1[4], wc, wa, rot;
  if ((m & 0x7fu) == 0x40u) {
    const uint32_t p0 = (uint32_t)(lo >> 63), p1 = (uint32_t)hi & 1u;
    const uint32_t j = bc7_index(lo, hi, 65u, 4u, slot);
    wc = wa = (64u * j + 7u) / 15u;
    rot = 0u;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      e0[c] = (bc7_bits(lo, hi, 7u + 14u * c, 7u) << 1) | p0;
      e1[c] = (bc7_bits(lo, hi, 14u + 14u * c, 7u) << 1) | p1;
    }
  } else if ((m & 0x3fu) == 0x20u) {
    rot = bc7_bits(lo, hi, 6u, 2u);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      e0[c] = bc7_expand(bc7_bits(lo, hi, 8u + 14u * c, 7u), 7u);
      e1[c] = bc7_expand(bc7_bits(lo, hi, 15u + 14u * c, 7u), 7u);
    }
    e0[3] = bc7_bits(lo, hi, 50u, 8u);
    e1[3] = bc7_bits(lo, hi, 58u, 8u);
    wc = (64u * bc7_index(lo, hi, 66u, 2u, slot) + 1u) / 3u;
    wa = (64u * bc7_index(lo, hi, 97u, 2u, slot) + 1u) / 3u;
  } else if ((m & 0x1fu) == 0x10u) {
    rot = bc7_bits(lo, hi, 5u, 2u);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      e0[c] = bc7_expand(bc7_bits(lo, hi, 8u + 10u * c, 5u), 5u);
      e1[c] = bc7_expand(bc7_bits(lo, hi, 13u + 10u * c, 5u), 5u);
    }
    e0[3] = bc7_expand(bc7_bits(lo, hi, 38u, 6u), 6u);
    e1[3] = bc7_expand(bc7_bits(lo, hi, 44u, 6u), 6u);
    const uint32_t w2 = (64u * bc7_index(lo, hi, 50u, 2u, slot) + 1u) / 3u;
    const uint32_t w3 = (64u * bc7_index(lo, hi, 81u, 3u, slot) + 3u) / 7u;
    const bool sel = (lo >> 7) & 1u;
    wc = sel ? w3 : w2;
    wa = sel ? w2 : w3;
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = 0.0f;
    return;
  }
  uint32_t t[4];
#pragma unroll
  for (int c = 0; c < 3; ++c) t[c] = ((64u - wc) * e0[c] + wc * e1[c] + 32u) >> 6;
  t[3] = ((64u - wa) * e0[3] + wa * e1[3] + 32u) >> 6;
  if (rot) {
    const uint32_t r = rot - 1u;
    const uint32_t x = r == 0u ? t[0] : (r == 1u ? t[1] : t[2]);
    t[0] = r == 0u ? t[3] : t[0];
    t[1] = r == 1u ? t[3] : t[1];
    t[2] = r == 2u ? t[3] : t[2];
    t[3] = x;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) v[c] = (float)t[c];
}

// Four channels (0..255) of texel `slot` of a footprint: 32 bytes of BC4 (codec 0) or one
// 16-byte BC7 block of mode 4, 5 or 6 (codec 1).
__device__ __forceinline__ void fp4(const uint8_t* fp, int codec, uint32_t slot, float v[4]) {
  if (codec) bc7_fp4_regs(*(const u4v*)fp, slot, v);
  else bc4_fp4(fp, slot, v);
}

// Standalone decode of BC7 blocks (the texel decode the hybrid kernels use), 16
// texels x 4 channels per block: out[64 b + 4 s + c].
__global__ __launch_bounds__(256) void k_bc7_blocks(const uint8_t* __restrict__ blocks, int64_t n,
                                                     uint8_t* __restrict__ out) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n; b += (int64_t)gridDim.x * blockDim.x) {
    const u4v blk = ((const u4v*)blocks)[b];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      uint32_t w[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        float v[4];
        bc7_fp4_regs(blk, (uint32_t)(4 * q + k), v);
        w[k] = (uint32_t)v[0] | (uint32_t)v[1] << 8 | (uint32_t)v[2] << 16 | (uint32_t)v[3] << 24;
      }
      ((u4v*)out)[4 * b + q] = (u4v){w[0], w[1], w[2], w[3]};
    }
  }
}

// Bilinear sample (4 channels, values / 255) of a block-compressed map of bw footprints per
// row starting at `base` (fpb bytes per footprint), accumulated into x with weight ws.
__device__ __forceinline__ void bc_bilinear4(const uint8_t* base, uint32_t bw, uint32_t fpb, int codec,
                                             const Axis& ax, const Axis& ay, float ws, float x[4]) {
  float w[4];
  tap_weights(ax, ay, w);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const uint32_t y = (uint32_t)((i & 2) ? ay.i1 : ay.i0), xx = (uint32_t)((i & 1) ? ax.i1 : ax.i0);
    float v[4];
    fp4(base + ((y >> 2) * bw + (xx >> 2)) * fpb, codec, 4u * (y & 3u) + (xx & 3u), v);
    const float wi = ws * w[i] * (1.0f / 255.0f);
#pragma unroll
    for (int c = 0; c < 4; ++c) x[c] = fmaf(wi, v[c], x[c]);
  }
}

// Two-channel 8-bit plane [N][size][2] sampled at coordinate c (texel centres) and rows k.
__device__ __forceinline__ void plane2(const uint8_t* p, int size, const Axis& a, const NodeT& k, float& r0,
                                       float& r1) {
  const uint16_t* q = (const uint16_t*)p;
  r0 = r1 = 0.0f;
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    const uint32_t row = (uint32_t)(kk ? k.i1 : k.i0) * (uint32_t)size;
    const float wk = (kk ? k.w1 : k.w0) * (1.0f / 255.0f);
#pragma unroll
    for (int aa = 0; aa < 2; ++aa) {
      const uint32_t v = q[row + (uint32_t)(aa ? a.i1 : a.i0)];
      const float w = wk * (aa ? a.w1 : a.w0);
      r0 = fmaf(w, (float)(v & 0xffu), r0);
      r1 = fmaf(w, (float)(v >> 8), r1);
    }
  }
}

// The 16 decoder inputs of an explicit query, as four chunks (CD: the codec, fixed per
// launch so that each instance carries one block decoder).
template <int CD>
__device__ __forceinline__ void hyb_query_feats(const ndgi_hybrid_model& m, float u, float v, const HybTime& ht,
                                                float r[4][4]) {
#pragma unroll
  for (int c = 0; c < 4; ++c) r[0][c] = r[1][c] = 0.0f;
  const Axis gx = coord_axis(u, m.Gu), gy = coord_axis(v, m.Gv);
  constexpr uint32_t fpb = CD ? 16u : 32u;
  const uint32_t gbw = (uint32_t)m.Gu >> 2, slice = gbw * ((uint32_t)m.Gv >> 2) * fpb;
  bc_bilinear4(m.fuvt + (uint32_t)ht.s.i0 * slice, gbw, fpb, CD, gx, gy, ht.s.w0, r[0]);
  bc_bilinear4(m.fuvt + (uint32_t)ht.s.i1 * slice, gbw, fpb, CD, gx, gy, ht.s.w1, r[0]);
  bc_bilinear4(m.fuv, (uint32_t)m.W >> 2, fpb, CD, coord_axis(u, m.W), coord_axis(v, m.H), 1.0f, r[1]);
  plane2(m.fut, m.U, coord_axis(u, m.U), ht.k, r[2][0], r[2][1]);
  plane2(m.fvt, m.V, coord_axis(v, m.V), ht.k, r[2][2], r[2][3]);
#pragma unroll
  for (int c = 0; c < 4; ++c) r[3][c] = ht.g[c];
}

// Descriptor ranges (host and device: page requests carry descriptors in device memory).
__host__ __device__ inline bool hybrid_ok(const ndgi_hybrid_model& m) {
  const bool dims = m.W >= 4 && m.H >= 4 && m.W <= 16384 && m.H <= 16384 && (m.W & 3) == 0 && (m.H & 3) == 0 &&
                    m.Gu >= 4 && m.Gv >= 4 && m.Gu <= m.W && m.Gv <= m.H && (m.Gu & 3) == 0 && (m.Gv & 3) == 0 &&
                    m.S >= 1 && m.S <= 1024 && m.U >= 1 && m.U <= m.W && m.V >= 1 && m.V <= m.H && m.Tt >= 1 &&
                    m.Tt <= 1024;
  const bool kinds = (m.hidden == 16 || m.hidden == 64) &&
                     (m.mlp_dtype == NDGI_DTYPE_F32 || m.mlp_dtype == NDGI_DTYPE_F16) &&
                     (m.n_keys == 0 || (m.n_keys >= 2 && m.n_keys <= NDGI_HYBRID_MAX_KEYS)) &&
                     (m.codec == NDGI_CODEC_BC4 || m.codec == NDGI_CODEC_BC7);
  const bool bufs = m.fuv && m.fuvt && m.fut && m.fvt && m.mlp && (m.n_keys == 0 || m.keys);
  // F_uvt offsets are 32-bit: S * Gu * Gv * (2 or 1) bytes below 4 GiB
  return dims && kinds && bufs && (uint64_t)m.S * (uint64_t)m.Gu * (uint64_t)m.Gv * 2u < (1ull << 32);
}

// ---------------------------------------------------------------------- query decode
// Grid-stride passes of 64 consecutive queries per wave (one query per lane in the feature
// phase, the decoder after the handoff); the decoder table and the key table are built
// once per workgroup in LDS.
template <int PREC, int HD, int CD>
__global__ __launch_bounds__(256) void k_hybrid_query(ndgi_hybrid_model m, const float* __restrict__ uvt, int64_t n,
                                                       void* __restrict__ out) {
  __shared__ HybTab<HD> tab;
  __shared__ float keys[NDGI_HYBRID_MAX_KEYS];
  hyb_build<PREC, HD>(tab, m.mlp, m.mlp_dtype);
  for (int i = threadIdx.x; i < m.n_keys; i += 256) keys[i] = m.keys[i];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t passes = (n + 63) >> 6;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  for (int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); p < passes; p += nwaves) {
    const int64_t mine = (p << 6) + lane;
    const int64_t qi = mine < n ? mine : n - 1;
    float u = uvt[qi * 3 + 0], v = uvt[qi * 3 + 1], t = uvt[qi * 3 + 2];
    const bool bad = !(isfinite(u) && isfinite(v) && isfinite(t));
    if (bad) u = v = t = 0.0f;
    const HybTime ht = hyb_time(m, t, [&](int i) { return keys[i]; });
    float r[4][4];
    hyb_query_feats<CD>(m, u, v, ht, r);
    const f4v acc = hyb_decode<PREC, HD>(tab, r, lane);
    if (mine < n) store_lin<PREC>(out, (size_t)mine, acc, bad);
  }
}

// ---------------------------------------------------------------------- page decode
// A request writes a region of (page + 2b)^2 texels (b = border); region texel i stands
// for map texel mirror(page * px - b + i), so the border repeats the neighbouring texels
// inside the map and mirrors the map past its edges.  The region is cut into side x side
// sub-tiles of at most 34 x 34 texels (side = ceil(region / 34): a 128 page is 4 x 4
// sub-tiles of 32^2, a 136 region with a 4-texel border 4 x 4 of 34^2), and a work item
// is (request, sub-tile), one workgroup per item over a persistent grid.  Per item the
// workgroup stages in LDS:
//  * the F_uvt nodes the sub-tile reads, decoded from both slices around tau and blended
//    in time (at most 35 x 35 nodes, since Gu <= W and Gv <= H);
//  * per sub-tile column: its F_uvt taps and weight and its V_ut (F_ut blended in time,
//    then along u); per row: its F_uvt taps and weight and its V_vt;
// then each pass of a wave decodes 64 consecutive texels of the sub-tile (row-major): the
// F_uv texel straight from its block (at a texel centre the bilinear weights are 1 and
// 0), the rest from LDS.  Texel-centre axes use exact integer arithmetic (texel_axis).
constexpr int kHybSub = 34;
constexpr int kHybWin = kHybSub + 1;

// Mirror addressing of a texel index on n texels (one reflection: -n <= i < 2n).
__device__ __forceinline__ int mirror_texel(int i, int n) { return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i); }

// Map-texel span [lo, hi] of region positions a..e (a <= e) under mirror addressing.
__device__ __forceinline__ void mirror_span(int a, int e, int n, int& lo, int& hi) {
  const int fa = mirror_texel(a, n), fe = mirror_texel(e, n);
  lo = a < 0 ? 0 : min(fa, fe);
  hi = e >= n ? n - 1 : max(fa, fe);
}

// Plane value (2 channels, / 255) of an 8-bit [N][size][2] plane at axis a, time rows k:
// blended in time first, then along the axis.
__device__ __forceinline__ float2 plane_at(const uint16_t* pl, uint32_t size, const Axis& a, const NodeT& k) {
  const uint32_t q00 = pl[(uint32_t)k.i0 * size + (uint32_t)a.i0], q01 = pl[(uint32_t)k.i1 * size + (uint32_t)a.i0];
  const uint32_t q10 = pl[(uint32_t)k.i0 * size + (uint32_t)a.i1], q11 = pl[(uint32_t)k.i1 * size + (uint32_t)a.i1];
  const float2 v0 = make_float2(fmaf(k.w1, (float)(q01 & 0xffu), k.w0 * (float)(q00 & 0xffu)) * (1.0f / 255.0f),
                                fmaf(k.w1, (float)(q01 >> 8), k.w0 * (float)(q00 >> 8)) * (1.0f / 255.0f));
  const float2 v1 = make_float2(fmaf(k.w1, (float)(q11 & 0xffu), k.w0 * (float)(q10 & 0xffu)) * (1.0f / 255.0f),
                                fmaf(k.w1, (float)(q11 >> 8), k.w0 * (float)(q10 >> 8)) * (1.0f / 255.0f));
  return make_float2(fmaf(a.w1, v1.x, a.w0 * v0.x), fmaf(a.w1, v1.y, a.w0 * v0.y));
}

template <int PREC, int HD>
__global__ __launch_bounds__(256) void k_hybrid_pages(const ndgi_hybrid_model* __restrict__ models, int32_t n_models,
                                                       const ndgi_page_req* __restrict__ reqs,
                                                       const int32_t* __restrict__ n_reqs_dev, int32_t max_reqs,
                                                       int32_t page, void* __restrict__ dst, int64_t pitch,
                                                       int32_t widths, int32_t border, uint32_t* __restrict__ flags) {
  __shared__ HybTab<HD> tab;
  __shared__ f4v win[kHybWin * kHybWin];
  __shared__ float skeys[NDGI_HYBRID_MAX_KEYS];
  __shared__ int4 rows_g[kHybSub], cols_g[kHybSub];     // F_uvt window taps and weight
  __shared__ float2 rows_v[kHybSub], cols_u[kHybSub];   // V_vt per row, V_ut per column
  static_assert(NDGI_HYBRID_MAX_KEYS <= 256, "one key per thread");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int n_req = *n_reqs_dev;
  n_req = n_req < 0 ? 0 : (n_req > max_reqs ? max_reqs : n_req);
  const int reg = page + 2 * border;                    // output region side
  const int side = (reg + kHybSub - 1) / kHybSub;
  const int sub = (reg + side - 1) / side;              // sub-tile side, <= kHybSub
  const int64_t per_req = (int64_t)side * side;
  const int64_t total = (int64_t)n_req * per_req;
  // each workgroup takes a contiguous run of items (equal cost), so consecutive items
  // mostly share a request and its decoder table
  const int64_t chunk = (total + gridDim.x - 1) / gridDim.x;
  const int64_t it_end = min(total, ((int64_t)blockIdx.x + 1) * chunk);
  int cur = -1;
  for (int64_t it = (int64_t)blockIdx.x * chunk; it < it_end; ++it) {
    const int r = (int)(it / per_req), s = (int)(it - (int64_t)r * per_req);
    const ndgi_page_req rq = reqs[r];
    bool ok = rq.model >= 0 && rq.model < n_models && rq.page_x >= 0 && rq.page_y >= 0;
    ndgi_hybrid_model m = {};
    if (ok) m = models[rq.model];
    ok = ok && hybrid_ok(m) && (int64_t)page * (rq.page_x + 1) <= m.W && (int64_t)page * (rq.page_y + 1) <= m.H &&
         (widths & (m.hidden == 16 ? 1 : 2)) != 0;
    if (!ok) {
      if (threadIdx.x == 0 && s == 0) atomicOr(flags, NDGI_FLAG_BAD_PAGE_REQUEST);
      continue;
    }
    if (m.hidden != HD) continue;   // served by the launch of the other width
    __syncthreads();                // the previous item's readers of the table and windows are done
    if (rq.model != cur) {          // new model: its decoder table and key times into LDS
      hyb_build<PREC, HD>(tab, m.mlp, m.mlp_dtype);
      if ((int)threadIdx.x < m.n_keys) skeys[threadIdx.x] = m.keys[threadIdx.x];
      cur = rq.model;
      __syncthreads();
    }
    const bool bad_t = !isfinite(rq.t);
    const HybTime ht = hyb_time(m, bad_t ? 0.0f : rq.t, [&](int i) { return skeys[i]; });
    // region origin of the sub-tile, its extent inside the region, the map position of
    // region texel 0 and the sub-tile's map-texel spans
    const int i0 = (s % side) * sub, j0 = (s / side) * sub;
    const int ni = min(sub, reg - i0), nj = min(sub, reg - j0);
    const int mx0 = page * rq.page_x - border, my0 = page * rq.page_y - border;
    int xlo, xhi, ylo, yhi;
    mirror_span(mx0 + i0, mx0 + i0 + ni - 1, m.W, xlo, xhi);
    mirror_span(my0 + j0, my0 + j0 + nj - 1, m.H, ylo, yhi);
    // node spans of the sub-tile; clamped to the LDS window (never reached when Gu <= W)
    const int wx0 = texel_axis<false>(xlo, m.Gu, m.W).i0, wy0 = texel_axis<false>(ylo, m.Gv, m.H).i0;
    const int nwx = min(texel_axis<false>(xhi, m.Gu, m.W).i1 - wx0 + 1, kHybWin);
    const int nwy = min(texel_axis<false>(yhi, m.Gv, m.H).i1 - wy0 + 1, kHybWin);
    {
      const uint32_t fpb = m.codec ? 16u : 32u;
      const uint32_t gbw = (uint32_t)m.Gu >> 2, slice = gbw * ((uint32_t)m.Gv >> 2) * fpb;
      const uint8_t* s0 = m.fuvt + (uint32_t)ht.s.i0 * slice;
      const uint8_t* s1 = m.fuvt + (uint32_t)ht.s.i1 * slice;
      for (int idx = threadIdx.x; idx < nwx * nwy; idx += 256) {
        const uint32_t gy = (uint32_t)(wy0 + idx / nwx), gx = (uint32_t)(wx0 + idx % nwx);
        const uint32_t off = ((gy >> 2) * gbw + (gx >> 2)) * fpb, slot = 4u * (gy & 3u) + (gx & 3u);
        float a[4], b[4];
        fp4(s0 + off, m.codec, slot, a);
        fp4(s1 + off, m.codec, slot, b);
        f4v o;
#pragma unroll
        for (int c = 0; c < 4; ++c) o[c] = fmaf(ht.s.w1, b[c], ht.s.w0 * a[c]) * (1.0f / 255.0f);
        win[idx] = o;
      }
      // threads 0..sub-1: the sub-tile's columns; 64..64+sub-1: its rows
      const int t = threadIdx.x;
      if (t < sub || (t >= 64 && t - 64 < sub)) {
        const bool isc = t < 64;
        const int k = isc ? t : t - 64;
        const int n = isc ? m.W : m.H, g = isc ? m.Gu : m.Gv, pn = isc ? m.U : m.V;
        const int pos = mirror_texel(isc ? mx0 + i0 + min(k, ni - 1) : my0 + j0 + min(k, nj - 1), n);
        const Axis a = texel_axis<false>(pos, g, n);
        const int o0 = isc ? wx0 : wy0, nn = isc ? nwx : nwy;
        const int4 e = make_int4(min(max(a.i0 - o0, 0), nn - 1), min(max(a.i1 - o0, 0), nn - 1), __float_as_int(a.w1), 0);
        const float2 pv = plane_at((const uint16_t*)(isc ? m.fut : m.fvt), (uint32_t)pn, texel_axis<false>(pos, pn, n),
                                   ht.k);
        if (isc) {
          cols_g[k] = e;
          cols_u[k] = pv;
        } else {
          rows_g[k] = e;
          rows_v[k] = pv;
        }
      }
    }
    __syncthreads();                // table and windows complete
    const uint32_t fbw = (uint32_t)m.W >> 2;
    const uint32_t ffb = m.codec ? 16u : 32u;
    const int nt = ni * nj, passes = (nt + 63) >> 6;
    const uint32_t mag = (65536u + (uint32_t)ni - 1u) / (uint32_t)ni;   // t / ni = (t * mag) >> 16 for t < 2^11
    // texel of pass p for this lane (row-major in the sub-tile; the tail repeats the last)
    auto texel_of = [&](int p, int& rj, int& ci) {
      const int tt = min(p * 64 + lane, nt - 1);
      rj = (int)(((uint32_t)tt * mag) >> 16);
      ci = tt - rj * ni;
    };
    // its F_uv footprint (one 16-byte BC7 block or 32 bytes of BC4) and texel slot
    auto footprint = [&](int rj, int ci, uint32_t& slot) {
      const int x = mirror_texel(mx0 + i0 + ci, m.W), y = mirror_texel(my0 + j0 + rj, m.H);
      slot = 4u * (uint32_t)(y & 3) + (uint32_t)(x & 3);
      return (const u4v*)(m.fuv + ((uint32_t)(y >> 2) * fbw + (uint32_t)(x >> 2)) * ffb);
    };
    // the F_uv footprint of the next pass is loaded while this one decodes
    int nr, nc;
    uint32_t nslot;
    texel_of(wave, nr, nc);
    const u4v* nfp = footprint(nr, nc, nslot);
    u4v fa = nfp[0], fb = m.codec ? fa : nfp[1];
    for (int p = wave; p < passes; p += 4) {
      const int rj = nr, ci = nc;
      const uint32_t slot = nslot;
      const u4v ca = fa, cb = fb;
      if (p + 4 < passes) {
        texel_of(p + 4, nr, nc);
        nfp = footprint(nr, nc, nslot);
        fa = nfp[0];
        fb = m.codec ? fa : nfp[1];
      }
      float rr[4][4];
      // V_uvt: bilinear over the staged nodes
      const int4 ag = rows_g[rj], cg = cols_g[ci];
      const float gyw1 = __int_as_float(ag.z), gxw1 = __int_as_float(cg.z), gxw0 = 1.0f - gxw1;
      const f4v c00 = win[ag.x * nwx + cg.x], c01 = win[ag.x * nwx + cg.y];
      const f4v c10 = win[ag.y * nwx + cg.x], c11 = win[ag.y * nwx + cg.y];
      const float w[4] = {(1.0f - gyw1) * gxw0, (1.0f - gyw1) * gxw1, gyw1 * gxw0, gyw1 * gxw1};
#pragma unroll
      for (int c = 0; c < 4; ++c) rr[0][c] = fmaf(w[3], c11[c], fmaf(w[2], c10[c], fmaf(w[1], c01[c], w[0] * c00[c])));
      // V_uv: the texel itself
      float sv[4];
      if (m.codec) bc7_fp4_regs(ca, slot, sv);
      else bc4_fp4_regs(ca, cb, slot, sv);
#pragma unroll
      for (int c = 0; c < 4; ++c) rr[1][c] = sv[c] * (1.0f / 255.0f);
      // V_ut (per column), V_vt (per row)
      const float2 vut = cols_u[ci], vvt = rows_v[rj];
      rr[2][0] = vut.x;
      rr[2][1] = vut.y;
      rr[2][2] = vvt.x;
      rr[2][3] = vvt.y;
#pragma unroll
      for (int c = 0; c < 4; ++c) rr[3][c] = ht.g[c];
      const f4v acc = hyb_decode<PREC, HD>(tab, rr, lane);
      if (p * 64 + lane < nt)
        store_lin<PREC>(dst, (size_t)(rq.dst_offset + (int64_t)(j0 + rj) * pitch + (i0 + ci)), acc, bad_t);
    }
  }
}

// ---------------------------------------------------------------------- host side
int check_hybrid(const ndgi_hybrid_model* m, const char* who) {
  if (!m) return fail(NDGI_ERR_INVALID_ARG, "%s: model is NULL", who);
  if (!hybrid_ok(*m))
    return fail(NDGI_ERR_INVALID_ARG,
                "%s: hybrid descriptor out of range (W %d H %d Gu %d Gv %d S %d U %d V %d Tt %d hidden %d "
                "mlp_dtype %d n_keys %d, or a NULL buffer)",
                who, m->W, m->H, m->Gu, m->Gv, m->S, m->U, m->V, m->Tt, m->hidden, m->mlp_dtype, m->n_keys);
  return NDGI_OK;
}

// Import of a block-compressed 4-channel map into a directly parameterised training state:
// texel (x, y) of slice sl becomes w[((sl H + y) W + x) 4 + c] = byte / 255 (FP32 division),
// the byte being the texel decode of the model's blocks (codec 0: 32 bytes of BC4 per
// footprint, codec 1: one BC7 block of mode 4, 5 or 6).
__global__ __launch_bounds__(256) void k_import_map(const uint8_t* __restrict__ blocks, int codec, int W, int H,
                                                     int64_t texels, float* __restrict__ w) {
  const int64_t per = (int64_t)W * H;
  const int fpb = codec ? 16 : 32;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < texels; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sl = i / per, rem = i - sl * per;
    const int x = (int)(rem % W), y = (int)(rem / W);
    const int64_t f = (sl * (H >> 2) + (y >> 2)) * (W >> 2) + (x >> 2);
    float v[4];
    fp4(blocks + f * fpb, codec, (uint32_t)(4 * (y & 3) + (x & 3)), v);
    *(float4*)(w + i * 4) = make_float4(v[0] / 255.0f, v[1] / 255.0f, v[2] / 255.0f, v[3] / 255.0f);
  }
}

int launch_import_map(const uint8_t* blocks, int codec, int W, int H, int S, float* w, int n_cu, hipStream_t s) {
  const int64_t texels = (int64_t)W * H * S;
  const int64_t want = (texels + 255) / 256, cap = (int64_t)n_cu * 16;
  hipLaunchKernelGGL(k_import_map, dim3((unsigned)(want < cap ? (want < 1 ? 1 : want) : cap)), dim3(256), 0, s, blocks,
                     codec, W, H, texels, w);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

int launch_bc7_blocks(const uint8_t* blocks, int64_t n, uint8_t* out, hipStream_t s) {
  const int64_t want = (n + 255) / 256;
  const int grid = (int)(want < 65536 ? want : 65536);
  hipLaunchKernelGGL(k_bc7_blocks, dim3(grid), dim3(256), 0, s, blocks, n, out);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

int launch_hybrid_query(ndgi_ctx* ctx, const ndgi_hybrid_model& m, const float* uvt, int64_t n, void* out, int prec,
                        hipStream_t s) {
  if (n == 0) return NDGI_OK;
  const int64_t want = ((n + 63) / 64 + 3) / 4;
#define NDGI_HQ(P, HD, CD)                                                                       \
  do {                                                                                           \
    int64_t wgs = resident_wgs(ctx, (const void*)k_hybrid_query<P, HD, CD>);                     \
    if (wgs > want) wgs = want;                                                                  \
    hipLaunchKernelGGL((k_hybrid_query<P, HD, CD>), dim3((unsigned)wgs), dim3(256), 0, s, m, uvt, n, out); \
  } while (0)
#define NDGI_HQ_CD(P, HD)                  \
  do {                                     \
    if (m.codec == NDGI_CODEC_BC7)         \
      NDGI_HQ(P, HD, NDGI_CODEC_BC7);      \
    else                                   \
      NDGI_HQ(P, HD, NDGI_CODEC_BC4);      \
  } while (0)
  if (prec == NDGI_PREC_F16) {
    if (m.hidden == 16) NDGI_HQ_CD(NDGI_PREC_F16, 16);
    else NDGI_HQ_CD(NDGI_PREC_F16, 64);
  } else {
    if (m.hidden == 16) NDGI_HQ_CD(NDGI_PREC_F32, 16);
    else NDGI_HQ_CD(NDGI_PREC_F32, 64);
  }
#undef NDGI_HQ_CD
#undef NDGI_HQ
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

int launch_hybrid_pages(ndgi_ctx* ctx, const ndgi_hybrid_model* models, int32_t n_models, const ndgi_page_req* reqs,
                        const int32_t* n_reqs, int32_t max_reqs, int32_t page, void* dst, int64_t pitch, int prec,
                        int32_t widths, int32_t border, hipStream_t s) {
  // one launch per decoder width present; each skips the requests of the other
  if (widths == 0) widths = 3;
#define NDGI_HP(P, HD)                                                                                           \
  hipLaunchKernelGGL((k_hybrid_pages<P, HD>), dim3(resident_wgs(ctx, (const void*)k_hybrid_pages<P, HD>)), dim3(256), \
                     0, s, models, n_models, reqs, n_reqs, max_reqs, page, dst, pitch, widths, border, ctx->flags_dev)
  if (prec == NDGI_PREC_F16) {
    if (widths & 1) NDGI_HP(NDGI_PREC_F16, 16);
    if (widths & 2) NDGI_HP(NDGI_PREC_F16, 64);
  } else {
    if (widths & 1) NDGI_HP(NDGI_PREC_F32, 16);
    if (widths & 2) NDGI_HP(NDGI_PREC_F32, 64);
  }
#undef NDGI_HP
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

}  // namespace ndgi
