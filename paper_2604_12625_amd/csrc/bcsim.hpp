// Block-parameterised feature maps of the hybrid layout (Sec. 3.4, Eq. 6-7): the texel
// value of a 4x4 footprint's endpoints and per-texel weights, continuous (the paper's BC
// simulation), rounded to a block format's grid (BC4 per channel or BC7 mode 6), or, for a
// directly optimised map, the texel values themselves; with the derivatives the training
// backward needs.  Shared by the training kernel and the export encoders.
#pragma once
#include "device.hpp"

namespace ndgi {

// One 4-channel texel of a block-parameterised map: ep = the footprint's [4][2] endpoints,
// w = the texel's 4 weights.  Rounded (bcsim): E = rint(fl32(255 e)), J = rint(fl32(7 w)),
// value floor(((7-J) E1 + J E2 + 3) / 7) / 255 and the straight-through derivatives of
// Eq. 7 at (E/255, J/7); otherwise Eq. 7 itself.
struct BcTex { float v[4], d1[4], d2[4], dw[4]; };
__device__ __forceinline__ BcTex bc_texel(const float* __restrict__ ep, const float* __restrict__ w, bool bcsim) {
#pragma clang fp contract(off)
  BcTex r;
  const float4 ea = *(const float4*)ep, eb = *(const float4*)(ep + 4);
  const float4 wv = *(const float4*)w;
  const float e1[4] = {ea.x, ea.z, eb.x, eb.z}, e2[4] = {ea.y, ea.w, eb.y, eb.w}, ww[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (bcsim) {
      const int E1 = (int)rintf(255.0f * e1[c]), E2 = (int)rintf(255.0f * e2[c]), J = (int)rintf(7.0f * ww[c]);
      r.v[c] = (float)(((7 - J) * E1 + J * E2 + 3) / 7) * (1.0f / 255.0f);
      r.d1[c] = (float)(7 - J) * (1.0f / 7.0f);
      r.d2[c] = (float)J * (1.0f / 7.0f);
      r.dw[c] = (float)(E2 - E1) * (1.0f / 255.0f);
    } else {
      r.v[c] = (1.0f - ww[c]) * e1[c] + ww[c] * e2[c];
      r.d1[c] = 1.0f - ww[c];
      r.d2[c] = ww[c];
      r.dw[c] = e2[c] - e1[c];
    }
  }
  return r;
}

// The same for the BC7 simulation (codec 1): one weight w per texel shared by the 4
// channels.  Each endpoint takes the 7-bit values and p-bit of BC7 mode 6 nearest to
// x = fl32(255 e) in summed squared error (v = rint((x - p) / 2) clamped to 0..127, E = 2 v + p;
// ties keep p = 0; the errors are compared exactly, in FP64); J = rint(fl32(15 w)) with
// weight (64 J + 7) / 15 (the format's table); value ((64 - w) E1 + w E2 + 32) >> 6 / 255;
// straight-through derivatives of Eq. 7 at (E/255, w/64).  dw[c] is the channel's share of
// the shared weight's derivative.
__device__ __forceinline__ void bc7_endpoint(const float e[4], int E[4]) {
#pragma clang fp contract(off)
  double err[2] = {0.0, 0.0};
  int Ep[2][4];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const float x = 255.0f * e[c];
      const int v = min(max((int)rintf((x - (float)p) * 0.5f), 0), 127);
      Ep[p][c] = 2 * v + p;
      const double dd = (double)Ep[p][c] - (double)x;
      err[p] += dd * dd;
    }
  const int p = err[1] < err[0] ? 1 : 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) E[c] = p ? Ep[1][c] : Ep[0][c];
}

__device__ __forceinline__ BcTex bc7_texel(const float* __restrict__ ep, float w, bool bcsim) {
#pragma clang fp contract(off)
  BcTex r;
  const float4 ea = *(const float4*)ep, eb = *(const float4*)(ep + 4);
  const float e1[4] = {ea.x, ea.z, eb.x, eb.z}, e2[4] = {ea.y, ea.w, eb.y, eb.w};
  if (bcsim) {
    int E1[4], E2[4];
    bc7_endpoint(e1, E1);
    bc7_endpoint(e2, E2);
    const int J = (int)rintf(15.0f * w);
    const int wt = (64 * J + 7) / 15;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      r.v[c] = (float)(((64 - wt) * E1[c] + wt * E2[c] + 32) >> 6) * (1.0f / 255.0f);
      r.d1[c] = 1.0f - (float)wt * (1.0f / 64.0f);
      r.d2[c] = (float)wt * (1.0f / 64.0f);
      r.dw[c] = (float)(E2[c] - E1[c]) * (1.0f / 255.0f);
    }
  } else {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      r.v[c] = (1.0f - w) * e1[c] + w * e2[c];
      r.d1[c] = 1.0f - w;
      r.d2[c] = w;
      r.dw[c] = e2[c] - e1[c];
    }
  }
  return r;
}

// Texel of either codec: weights at w (4 per texel for BC4, 1 for BC7).  direct: the map is
// its texel values themselves (4 per texel, the BC4 layout), endpoints unused.
__device__ __forceinline__ BcTex sim_texel(const float* __restrict__ ep, const float* __restrict__ w, bool bcsim,
                                           bool direct, int codec) {
  if (direct) {
    BcTex r;
    const float4 wv = *(const float4*)w;
    const float ww[4] = {wv.x, wv.y, wv.z, wv.w};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      r.v[c] = ww[c];
      r.d1[c] = 0.0f;
      r.d2[c] = 0.0f;
      r.dw[c] = 1.0f;
    }
    return r;
  }
  return codec ? bc7_texel(ep, *w, bcsim) : bc_texel(ep, w, bcsim);
}

// Export reconstruction (Sec. 3.4, last paragraph of Feature Map Compression): the 8-bit
// texel (4 channels) of a block-parameterised map as training with `kind` reads it, before
// block compression.  kSrcRounded: the rounded simulation's byte (the texel of the exact
// export); kSrcDirect: the weight itself; kSrcLerp: the FP32 Eq. 7 lerp
// fl32(fl32(fl32(1 - w) e1) + fl32(w e2)); the last two quantised as rint(fl32(255 v))
// clamped to 0..255.  codec: the state's layout (1: one weight per texel).
enum { kSrcLerp = 0, kSrcRounded = 1, kSrcDirect = 2 };
__device__ __forceinline__ void map_texel_u8(const float* __restrict__ ep, const float* __restrict__ w, int kind,
                                             int codec, int q[4]) {
#pragma clang fp contract(off)
  const float4 ea = *(const float4*)ep, eb = *(const float4*)(ep + 4);
  const float e1[4] = {ea.x, ea.z, eb.x, eb.z}, e2[4] = {ea.y, ea.w, eb.y, eb.w};
  if (kind == kSrcRounded) {
    if (codec) {
      int E1[4], E2[4];
      bc7_endpoint(e1, E1);
      bc7_endpoint(e2, E2);
      const int J = (int)rintf(15.0f * w[0]);
      const int wt = (64 * J + 7) / 15;
#pragma unroll
      for (int c = 0; c < 4; ++c) q[c] = ((64 - wt) * E1[c] + wt * E2[c] + 32) >> 6;
    } else {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int E1 = (int)rintf(255.0f * e1[c]), E2 = (int)rintf(255.0f * e2[c]), J = (int)rintf(7.0f * w[c]);
        q[c] = ((7 - J) * E1 + J * E2 + 3) / 7;
      }
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float v;
    if (kind == kSrcDirect) {
      v = w[c];
    } else {
      const float wc = codec ? w[0] : w[c];
      v = (1.0f - wc) * e1[c] + wc * e2[c];
    }
    q[c] = min(max((int)rintf(__fmul_rn(255.0f, v)), 0), 255);
  }
}

}  // namespace ndgi
