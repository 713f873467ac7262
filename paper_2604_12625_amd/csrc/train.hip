// Training under BC simulation: fused forward / loss / backward, deterministic reduction
// of the decoder gradients, dense Adam, export to BC4, and tiled-PSNR statistics.
//
// Forward per 16-sample group (lane (g, j) = sample j, inputs 2g, 2g+1 of each map), as in
// the decoder but in FP32 MFMA (v_mfma_f32_16x16x4_f32) and with the BC-simulated spatial
// texel.  Backward chains dz -> dh2 -> dh1 -> dx with the transposed weights as the A
// operand, so each lane ends with d(loss)/d(its own four inputs) and scatters them to the
// endpoint, weight and grid gradients with float atomics.  Decoder weight gradients
// (sum over samples of outer products) run on MFMA with the samples as K: activations are
// staged through LDS to put hidden units on lanes.  Bias gradients are per-lane sums reduced
// across the wave with shuffles.  Each wave writes one partial row; a second kernel sums
// the rows in a fixed order.
#include "device.hpp"
#include "internal.hpp"

namespace ndgi {

constexpr int kPadU = 48;   // LDS row stride (floats) of 32-wide activations: rows g, g+1
                            // of one half-wave land on disjoint banks
constexpr int kPadX = 16;

struct TrainLds {
  float x[16 * kPadX];
  float h1[16 * kPadU];
  float h2[16 * kPadU];
  float d1[16 * kPadU];
  float d2[16 * kPadU];
  float dz[16 * 4];
};

// Slots of the per-lane weight table (see k_train).
constexpr int kSA1 = 0, kSA2 = 8, kSA3 = 24, kSW3T = 32, kSW2T = 34, kSW1T = 50, kSC1 = 58, kSC2 = 66,
              kSC3 = 74, kWSlots = 78;

__device__ __forceinline__ float half_bits(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }

struct TrainDims {
  int W, H, Gw, Gh, T;
  int64_t off_w, off_g, off_mlp;   // segment offsets in the flat arrays
};

template <int MODE, bool R4>
__global__ __launch_bounds__(256) void k_train(TrainDims d, const float* __restrict__ P, float* __restrict__ G,
                                                const uint32_t* __restrict__ samples, int64_t n,
                                                const uint16_t* __restrict__ target, float* __restrict__ pred,
                                                const float* __restrict__ grad_pred, float inv3n,
                                                float* __restrict__ partials, double* __restrict__ loss_part,
                                                uint32_t* __restrict__ flags) {
  __shared__ TrainLds lds_all[4];
  __shared__ float wsl[kWSlots][64];
  const int wave = threadIdx.x >> 6;
  TrainLds& L = lds_all[wave];
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, j = lane & 15;
  const float* ep = P;
  const float* wts = P + d.off_w;
  const float* grid = P + d.off_g;
  const float* mlp = P + d.off_mlp;
  float* g_ep = G;
  float* g_w = G + d.off_w;
  float* g_grid = G + d.off_g;

  // Forward weights (the FP32 decoder's A operands), transposed weights for the backward
  // pass and the biases in C layout, one float per lane per slot, staged in LDS once per
  // workgroup: held in registers they would leave room for one wave per SIMD only.
  for (int idx = threadIdx.x; idx < kWSlots * 64; idx += 256) {
    const int slot = idx >> 6, ln = idx & 63;
    const int gg = ln >> 4, ii = ln & 15;
    float v = 0.0f;
    if (slot < kSA2) {                       // a1[mc][e]
      const int mc = (slot - kSA1) >> 2, e = (slot - kSA1) & 3;
      v = mlp[kOffW1 + (16 * mc + ii) * 16 + input_of(gg, e)];
    } else if (slot < kSA3) {                // a2[mc][e]
      const int mc = (slot - kSA2) >> 3, e = (slot - kSA2) & 7;
      v = mlp[kOffW2 + (16 * mc + ii) * 32 + unit_of(gg, e)];
    } else if (slot < kSW3T) {               // a3 of output group 0: rows 0..2 at lanes i < 3
      const int e = slot - kSA3;
      v = ii < 3 ? mlp[kOffW3 + ii * 32 + unit_of(gg, e)] : 0.0f;
    } else if (slot < kSW2T) {               // w3t[mc]
      const int mc = slot - kSW3T;
      v = gg < 3 ? mlp[kOffW3 + gg * 32 + 16 * mc + ii] : 0.0f;
    } else if (slot < kSW1T) {               // w2t[mc][m]
      const int mc = (slot - kSW2T) >> 3, m = (slot - kSW2T) & 7;
      v = mlp[kOffW2 + unit_of(gg, m) * 32 + 16 * mc + ii];
    } else if (slot < kSC1) {                // w1t[m]
      const int m = slot - kSW1T;
      v = mlp[kOffW1 + unit_of(gg, m) * 16 + input_of(ii >> 2, ii & 3)];
    } else if (slot < kSC2) {                // c1[mc][r]
      const int mc = (slot - kSC1) >> 2, r = (slot - kSC1) & 3;
      v = mlp[kOffB1 + 16 * mc + 4 * gg + r];
    } else if (slot < kSC3) {                // c2[mc][r]
      const int mc = (slot - kSC2) >> 2, r = (slot - kSC2) & 3;
      v = mlp[kOffB2 + 16 * mc + 4 * gg + r];
    } else {                                 // c3[r]
      const int r = slot - kSC3;
      v = r < 3 ? mlp[kOffB3 + r] : 0.0f;
    }
    wsl[slot][ln] = v;
  }
  __syncthreads();
  auto W = [&](int slot) { return wsl[slot][lane]; };
  auto C4 = [&](int slot) { return f4v{W(slot), W(slot + 1), W(slot + 2), W(slot + 3)}; };

  f4v gW2[2][2], gW1[2], gW3[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    gW1[a] = gW3[a] = f4v{0, 0, 0, 0};
    gW2[a][0] = gW2[a][1] = f4v{0, 0, 0, 0};
  }
  float gb1[8], gb2[8], gb3 = 0.0f;
#pragma unroll
  for (int e = 0; e < 8; ++e) gb1[e] = gb2[e] = 0.0f;
  double loss = 0.0;

  const int64_t groups = (n + 15) >> 4;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  const int64_t wave_id = (int64_t)blockIdx.x * 4 + wave;
  // A group's sample words and gathered inputs are loaded one group ahead of their use (the
  // word two groups ahead), so that the loads a group waits for were issued before the
  // previous group's gradient atomics and its wait does not include them.
  struct GroupIn {
    bool valid;
    int x, y, k;
    float4 e4;       // (e1, e2) of channels 2g, 2g+1
    float2 w2;       // weights of channels 2g, 2g+1
    float2 gv[4];    // grid corners (yy, xx), channels 2g, 2g+1
    float tg[3];     // target RGB (lanes g = 0)
  };
  auto word_at = [&](int64_t grp) -> uint32_t {
    const int64_t s = (grp << 4) + j;
    return grp < groups && s < n ? samples[s] : 0u;
  };
  auto fetch = [&](int64_t grp, uint32_t word) {
    GroupIn in;
    const int64_t s = (grp << 4) + j;
    in.valid = grp < groups && s < n;
    int x = word & 0xfff, y = (word >> 12) & 0xfff, k = word >> 24;
    if (in.valid && (x >= d.W || y >= d.H || k >= d.T)) {
      in.valid = false;
      if (g == 0) atomicOr(flags, NDGI_FLAG_BAD_SAMPLE);
    }
    if (!in.valid) x = y = k = 0;
    in.x = x;
    in.y = y;
    in.k = k;
    const size_t blk = ((size_t)(y >> 2) * (d.W >> 2) + (x >> 2)) * 8 + 2 * g;
    in.e4 = *(const float4*)(ep + blk * 2);
    in.w2 = *(const float2*)(wts + ((size_t)y * d.W + x) * 8 + 2 * g);
    const Axis ax = texel_axis<R4>(x, d.Gw, d.W), ay = texel_axis<R4>(y, d.Gh, d.H);
#pragma unroll
    for (int yy = 0; yy < 2; ++yy)
#pragma unroll
      for (int xx = 0; xx < 2; ++xx) {
        const size_t node = ((size_t)k * d.Gh + (yy ? ay.i1 : ay.i0)) * d.Gw + (xx ? ax.i1 : ax.i0);
        in.gv[2 * yy + xx] = *(const float2*)(grid + node * 8 + 2 * g);
      }
    in.tg[0] = in.tg[1] = in.tg[2] = 0.0f;
    if constexpr (MODE == NDGI_TRAIN_LOSS_GRAD) {
      if (g == 0 && in.valid) {
        const uint16_t* tp = target + (((size_t)k * d.H + y) * d.W + x) * 3;
        in.tg[0] = half_bits(tp[0]);
        in.tg[1] = half_bits(tp[1]);
        in.tg[2] = half_bits(tp[2]);
      }
    }
    return in;
  };
  uint32_t word_next = word_at(wave_id + nwaves);
  GroupIn cur = fetch(wave_id, word_at(wave_id)), nxt;
  for (int64_t grp = wave_id; grp < groups; grp += nwaves, cur = nxt) {
    nxt = fetch(grp + nwaves, word_next);
    word_next = word_at(grp + 2 * nwaves);
    const int64_t s = (grp << 4) + j;
    const bool valid = cur.valid;
    const int x = cur.x, y = cur.y, k = cur.k;

    // ---- inputs: BC-simulated spatial texel (channels 2g, 2g+1) and grid at key k
    const size_t blk = ((size_t)(y >> 2) * (d.W >> 2) + (x >> 2)) * 8 + 2 * g;   // block-channel index
    const float4 e4 = cur.e4;
    const float2 w2 = cur.w2;
    const int E1a = (int)rintf(__fmul_rn(255.0f, e4.x)), E2a = (int)rintf(__fmul_rn(255.0f, e4.y));
    const int E1b = (int)rintf(__fmul_rn(255.0f, e4.z)), E2b = (int)rintf(__fmul_rn(255.0f, e4.w));
    const int Ja = (int)rintf(__fmul_rn(7.0f, w2.x)), Jb = (int)rintf(__fmul_rn(7.0f, w2.y));
    float f[4];
    f[0] = (float)(((7 - Ja) * E1a + Ja * E2a + 3) / 7) * (1.0f / 255.0f);
    f[1] = (float)(((7 - Jb) * E1b + Jb * E2b + 3) / 7) * (1.0f / 255.0f);
    const Axis ax = texel_axis<R4>(x, d.Gw, d.W), ay = texel_axis<R4>(y, d.Gh, d.H);
    {
      float a = 0.0f, b = 0.0f;
#pragma unroll
      for (int yy = 0; yy < 2; ++yy)
#pragma unroll
        for (int xx = 0; xx < 2; ++xx) {
          const float w = (yy ? ay.w1 : ay.w0) * (xx ? ax.w1 : ax.w0);
          const float2 v = cur.gv[2 * yy + xx];
          a = fmaf(w, v.x, a);
          b = fmaf(w, v.y, b);
        }
      f[2] = a;
      f[3] = b;
    }

    // ---- forward MLP
    f4v p0 = C4(kSC1), p1 = C4(kSC1 + 4);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      p0 = __builtin_amdgcn_mfma_f32_16x16x4f32(W(kSA1 + m), f[m], p0, 0, 0, 0);
      p1 = __builtin_amdgcn_mfma_f32_16x16x4f32(W(kSA1 + 4 + m), f[m], p1, 0, 0, 0);
    }
    float h1[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      h1[r] = fmaxf(p0[r], 0.0f);
      h1[4 + r] = fmaxf(p1[r], 0.0f);
    }
    f4v r0 = C4(kSC2), r1 = C4(kSC2 + 4);
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      r0 = __builtin_amdgcn_mfma_f32_16x16x4f32(W(kSA2 + m), h1[m], r0, 0, 0, 0);
      r1 = __builtin_amdgcn_mfma_f32_16x16x4f32(W(kSA2 + 8 + m), h1[m], r1, 0, 0, 0);
    }
    float h2[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      h2[r] = fmaxf(r0[r], 0.0f);
      h2[4 + r] = fmaxf(r1[r], 0.0f);
    }
    f4v z = C4(kSC3);   // output rows 0..2 of group 0's slot (lanes g = 0)
#pragma unroll
    for (int m = 0; m < 8; ++m) z = __builtin_amdgcn_mfma_f32_16x16x4f32(W(kSA3 + m), h2[m], z, 0, 0, 0);

    // ---- output, loss, dL/dz (lanes g = 0 own sample j's three channels)
    float dz0 = 0.0f, dz1 = 0.0f, dz2 = 0.0f;
    if (g == 0 && valid) {
      const float c0 = expf(z[0]), c1 = expf(z[1]), c2 = expf(z[2]);
      if constexpr (MODE == NDGI_TRAIN_FORWARD) {
        pred[s * 3 + 0] = c0;
        pred[s * 3 + 1] = c1;
        pred[s * 3 + 2] = c2;
      } else if constexpr (MODE == NDGI_TRAIN_BACKWARD) {
        dz0 = grad_pred[s * 3 + 0] * c0;
        dz1 = grad_pred[s * 3 + 1] * c1;
        dz2 = grad_pred[s * 3 + 2] * c2;
      } else {
        const float e0 = c0 - cur.tg[0], e1 = c1 - cur.tg[1], e2 = c2 - cur.tg[2];
        loss += (double)e0 * e0 + (double)e1 * e1 + (double)e2 * e2;
        dz0 = 2.0f * inv3n * e0 * c0;
        dz1 = 2.0f * inv3n * e1 * c1;
        dz2 = 2.0f * inv3n * e2 * c2;
        if (pred) {
          pred[s * 3 + 0] = c0;
          pred[s * 3 + 1] = c1;
          pred[s * 3 + 2] = c2;
        }
      }
    }
    if constexpr (MODE == NDGI_TRAIN_FORWARD) continue;

    // B operand of the output-layer backward: lane (g, j) takes channel g of sample j
    const float v0 = __shfl(dz0, j), v1 = __shfl(dz1, j), v2 = __shfl(dz2, j);
    const float dzb = g == 0 ? v0 : (g == 1 ? v1 : (g == 2 ? v2 : 0.0f));

    // ---- backward through the decoder
    f4v q0 = {0, 0, 0, 0}, q1 = {0, 0, 0, 0};
    q0 = __builtin_amdgcn_mfma_f32_16x16x4f32(W(kSW3T), dzb, q0, 0, 0, 0);
    q1 = __builtin_amdgcn_mfma_f32_16x16x4f32(W(kSW3T + 1), dzb, q1, 0, 0, 0);
    float d2[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      d2[r] = r0[r] > 0.0f ? q0[r] : 0.0f;
      d2[4 + r] = r1[r] > 0.0f ? q1[r] : 0.0f;
    }
    f4v t0 = {0, 0, 0, 0}, t1 = {0, 0, 0, 0};
#pragma unroll
    for (int m = 0; m < 8; ++m) {
      t0 = __builtin_amdgcn_mfma_f32_16x16x4f32(W(kSW2T + m), d2[m], t0, 0, 0, 0);
      t1 = __builtin_amdgcn_mfma_f32_16x16x4f32(W(kSW2T + 8 + m), d2[m], t1, 0, 0, 0);
    }
    float d1[8];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      d1[r] = p0[r] > 0.0f ? t0[r] : 0.0f;
      d1[4 + r] = p1[r] > 0.0f ? t1[r] : 0.0f;
    }
    f4v dx = {0, 0, 0, 0};
#pragma unroll
    for (int m = 0; m < 8; ++m) dx = __builtin_amdgcn_mfma_f32_16x16x4f32(W(kSW1T + m), d1[m], dx, 0, 0, 0);
    // dx[r] = dLoss/d(input_of(g, r)) of sample j

    // ---- scatter input gradients (straight-through BC simulation; grid corners)
    // A float atomic costs one memory request per 64-byte segment it touches, however many
    // of the segment's words its lanes add to.  Lane (g, j) holds the gradients of channels
    // 2g, 2g+1 of sample j, so atomics issued from there would cover 16 segments with four
    // words each.  The values are first moved between lanes so that each instruction covers
    // whole segments: the 16 endpoint words of 4 samples, the 8 weight words of 8 samples,
    // and the two adjacent grid nodes of one corner row (8 channels each) of 4 samples.  The
    // values and the words they go to are unchanged.
    {
      const float da = dx[0], db = dx[1];
      // straight-through derivatives 1 - J/7 and J/7, written (7 - J)/7 so that J = 7 gives
      // exactly 0 (1 - J * (1/7) contracts to an FMA that leaves -4e-8 there)
      const float ve0 = da * ((float)(7 - Ja) * (1.0f / 7.0f)), ve1 = da * ((float)Ja * (1.0f / 7.0f));
      const float ve2 = db * ((float)(7 - Jb) * (1.0f / 7.0f)), ve3 = db * ((float)Jb * (1.0f / 7.0f));
      const float vw0 = da * (float)(E2a - E1a) * (1.0f / 255.0f), vw1 = db * (float)(E2b - E1b) * (1.0f / 255.0f);
      const int ok_j = valid ? 1 : 0;
      const uint32_t block_j = (uint32_t)(blk >> 3), texel_j = (uint32_t)y * (uint32_t)d.W + (uint32_t)x;
      const uint32_t row0_j = (uint32_t)k * (uint32_t)d.Gh + (uint32_t)ay.i0;
      const uint32_t row1_j = (uint32_t)k * (uint32_t)d.Gh + (uint32_t)ay.i1;
      const int w16 = lane & 15, s4 = lane >> 4;   // word of a 16-word segment, sample of four
      // endpoints [block][channel][2]: word w of a block's 16 is channel w / 2, held by g = w / 4
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int src = (w16 >> 2) * 16 + 4 * r + s4;
        const float t0 = __shfl(ve0, src), t1 = __shfl(ve1, src), t2 = __shfl(ve2, src), t3 = __shfl(ve3, src);
        const uint32_t bq = __shfl(block_j, src);
        const int c = w16 & 3;
        if (__shfl(ok_j, src)) atomicAdd(g_ep + (size_t)bq * 16 + w16, c == 0 ? t0 : (c == 1 ? t1 : (c == 2 ? t2 : t3)));
      }
      // weights [texel][channel]: eight samples per instruction, channel w8 held by g = w8 / 2
      const int w8 = lane & 7, s8 = lane >> 3;
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int src = (w8 >> 1) * 16 + 8 * r + s8;
        const float t0 = __shfl(vw0, src), t1 = __shfl(vw1, src);
        const uint32_t tq = __shfl(texel_j, src);
        if (__shfl(ok_j, src)) atomicAdd(g_w + (size_t)tq * 8 + w8, (w8 & 1) ? t1 : t0);
      }
      // grid [key][row][column][channel]: per corner row, columns i0, i1 (8 channels each)
      const int ch = w16 & 7, xx = w16 >> 3;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int src = (ch >> 1) * 16 + 4 * r + s4;
        const float g2 = __shfl(dx[2], src), g3 = __shfl(dx[3], src);
        const float wx0 = __shfl(ax.w0, src), wx1 = __shfl(ax.w1, src);
        const float wy0 = __shfl(ay.w0, src), wy1 = __shfl(ay.w1, src);
        const int ix0 = __shfl(ax.i0, src), ix1 = __shfl(ax.i1, src);
        const uint32_t rq0 = __shfl(row0_j, src), rq1 = __shfl(row1_j, src);
        if (__shfl(ok_j, src)) {
          const float gv = (ch & 1) ? g3 : g2, wx = xx ? wx1 : wx0;
          const int ix = xx ? ix1 : ix0;
          atomicAdd(g_grid + ((size_t)rq0 * d.Gw + ix) * 8 + ch, (wy0 * wx) * gv);
          atomicAdd(g_grid + ((size_t)rq1 * d.Gw + ix) * 8 + ch, (wy1 * wx) * gv);
        }
      }
    }

    // ---- decoder weight gradients: stage activations with units on columns
    *(float2*)&L.x[j * kPadX + 2 * g] = make_float2(f[0], f[1]);
    *(float2*)&L.x[j * kPadX + 8 + 2 * g] = make_float2(f[2], f[3]);
    *(float4*)&L.h1[j * kPadU + 4 * g] = make_float4(h1[0], h1[1], h1[2], h1[3]);
    *(float4*)&L.h1[j * kPadU + 16 + 4 * g] = make_float4(h1[4], h1[5], h1[6], h1[7]);
    *(float4*)&L.h2[j * kPadU + 4 * g] = make_float4(h2[0], h2[1], h2[2], h2[3]);
    *(float4*)&L.h2[j * kPadU + 16 + 4 * g] = make_float4(h2[4], h2[5], h2[6], h2[7]);
    *(float4*)&L.d2[j * kPadU + 4 * g] = make_float4(d2[0], d2[1], d2[2], d2[3]);
    *(float4*)&L.d2[j * kPadU + 16 + 4 * g] = make_float4(d2[4], d2[5], d2[6], d2[7]);
    *(float4*)&L.d1[j * kPadU + 4 * g] = make_float4(d1[0], d1[1], d1[2], d1[3]);
    *(float4*)&L.d1[j * kPadU + 16 + 4 * g] = make_float4(d1[4], d1[5], d1[6], d1[7]);
    L.dz[j * 4 + g] = dzb;
    wave_sync();
    const int i = lane & 15;
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const int row = 4 * s4 + g;   // sample of this K step held by lane group g
      const float a_d2_0 = L.d2[row * kPadU + i], a_d2_1 = L.d2[row * kPadU + 16 + i];
      const float a_d1_0 = L.d1[row * kPadU + i], a_d1_1 = L.d1[row * kPadU + 16 + i];
      const float a_dz = i < 3 ? L.dz[row * 4 + i] : 0.0f;
      const float b_h1_0 = L.h1[row * kPadU + i], b_h1_1 = L.h1[row * kPadU + 16 + i];
      const float b_h2_0 = L.h2[row * kPadU + i], b_h2_1 = L.h2[row * kPadU + 16 + i];
      const float b_x = L.x[row * kPadX + i];
      gW2[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_d2_0, b_h1_0, gW2[0][0], 0, 0, 0);
      gW2[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_d2_0, b_h1_1, gW2[0][1], 0, 0, 0);
      gW2[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_d2_1, b_h1_0, gW2[1][0], 0, 0, 0);
      gW2[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_d2_1, b_h1_1, gW2[1][1], 0, 0, 0);
      gW1[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_d1_0, b_x, gW1[0], 0, 0, 0);
      gW1[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_d1_1, b_x, gW1[1], 0, 0, 0);
      gW3[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_dz, b_h2_0, gW3[0], 0, 0, 0);
      gW3[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_dz, b_h2_1, gW3[1], 0, 0, 0);
    }
    wave_sync();
    // ---- bias gradients: per-lane sums, reduced across the wave after the loop
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      gb1[e] += d1[e];
      gb2[e] += d2[e];
    }
    gb3 += dzb;
  }

  if constexpr (MODE == NDGI_TRAIN_FORWARD) return;
  // reduce bias partials over the 16 samples-lanes of each row (xor within 16 lanes)
#pragma unroll
  for (int off = 1; off < 16; off <<= 1) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      gb1[e] += __shfl_xor(gb1[e], off);
      gb2[e] += __shfl_xor(gb2[e], off);
    }
    gb3 += __shfl_xor(gb3, off);
  }
  float* out = partials + (size_t)wave_id * kPartialStride;
  const int i = lane & 15;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
#pragma unroll
    for (int mc = 0; mc < 2; ++mc) {
      const int u = 16 * mc + 4 * g + r;
      out[kOffW1 + u * 16 + i] = gW1[mc][r];
      out[kOffW2 + u * 32 + i] = gW2[mc][0][r];
      out[kOffW2 + u * 32 + 16 + i] = gW2[mc][1][r];
    }
    if (g == 0 && r < 3) {
      out[kOffW3 + r * 32 + i] = gW3[0][r];
      out[kOffW3 + r * 32 + 16 + i] = gW3[1][r];
    }
  }
  if (i == 0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      out[kOffB1 + unit_of(g, e)] = gb1[e];
      out[kOffB2 + unit_of(g, e)] = gb2[e];
    }
    if (g < 3) out[kOffB3 + g] = gb3;
  }
  // FP64 loss: wave reduction, one value per wave
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) loss += __shfl_xor(loss, off);
  if (lane == 0) loss_part[wave_id] = loss;
}

// First stage of the decoder-gradient reduction: workgroup (cb, rb) sums rows
// [rb * kRowBlock, (rb + 1) * kRowBlock) of the per-wave partial rows for 256 columns, in
// row order, into stage row rb.  Fixed order throughout, so the result is deterministic.
constexpr int kRowBlock = 64;
__global__ __launch_bounds__(256) void k_reduce_rows(const float* __restrict__ partials, int rows,
                                                      float* __restrict__ stage) {
  const int col = blockIdx.x * 256 + threadIdx.x;
  if (col >= NDGI_MLP_SIZE) return;
  const int r0 = blockIdx.y * kRowBlock, r1 = min(rows, r0 + kRowBlock);
  // all of the thread's loads in flight together, then summed in row order (rows past the
  // end add +0, which leaves a sum that started at +0 unchanged)
  float v[kRowBlock];
#pragma unroll
  for (int k = 0; k < kRowBlock; ++k) v[k] = r0 + k < r1 ? partials[(size_t)(r0 + k) * kPartialStride + col] : 0.0f;
  float acc = 0.0f;
#pragma unroll
  for (int k = 0; k < kRowBlock; ++k) acc += v[k];
  stage[(size_t)blockIdx.y * kPartialStride + col] = acc;
}

// Second stage: sum the stage rows into the decoder gradients (fixed order), and the loss
// parts into *loss_out.  One workgroup of 256 threads per 64 columns.
__global__ __launch_bounds__(256) void k_reduce_partials(const float* __restrict__ partials, int rows,
                                                          float* __restrict__ g_mlp, const double* __restrict__ loss_part,
                                                          int loss_rows, double scale, double* __restrict__ loss_out) {
  __shared__ float red[4][64];
  const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + c;
  float acc = 0.0f;
  if (col < NDGI_MLP_SIZE)
    for (int r = ph; r < rows; r += 4 * 8) {   // eight rows' loads in flight, summed in row order
      float v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = r + 4 * k < rows ? partials[(size_t)(r + 4 * k) * kPartialStride + col] : 0.0f;
#pragma unroll
      for (int k = 0; k < 8; ++k) acc += v[k];
    }
  red[ph][c] = acc;
  __syncthreads();
  if (ph == 0 && col < NDGI_MLP_SIZE) g_mlp[col] += ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
  if (blockIdx.x == 0 && loss_out) {
    __shared__ double lred[256];
    double l = 0.0;
    for (int r = threadIdx.x; r < loss_rows; r += 256 * 8) {   // eight loads in flight
      double v[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = r + 256 * k < loss_rows ? loss_part[r + 256 * k] : 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) l += v[k];
    }
    lred[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) lred[threadIdx.x] += lred[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) *loss_out = lred[0] * scale;
  }
}

typedef float nf4 __attribute__((ext_vector_type(4)));
constexpr int64_t kLlcBytes = 256ll << 20;   // MI355X last-level (Infinity) cache

// Dense Adam (bias-corrected, as torch.optim.Adam), projection of the BC parameters to
// [0, 1], gradient reset.  Four parameters per thread; segment boundaries are multiples of 4.
template <bool NT>
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ gr, float* __restrict__ m,
                                               float* __restrict__ v, int64_t n, int64_t off_g, int64_t off_mlp,
                                               float lr_feat, float lr_mlp, float b1, float b2, float eps,
                                               float step_feat, float step_mlp, float inv_sqrt_bc2) {
  const int64_t n4 = n >> 2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q <= n4; q += stride) {
    const int64_t i0 = q << 2;
    if (i0 >= n) break;
    const bool clampseg = i0 < off_g;
    const float ss = i0 < off_mlp ? step_feat : step_mlp;
    if (i0 + 4 <= n) {
      // NT: streaming (non-temporal) accesses for a state larger than the last-level cache, so
      // that its lines do not displace what the next gradient pass re-reads
      auto ld = [&](const float* q) {
        return NT ? __builtin_nontemporal_load((const nf4*)q) : *(const nf4*)q;
      };
      auto st = [&](float* q, nf4 x) {
        if constexpr (NT) __builtin_nontemporal_store(x, (nf4*)q);
        else *(nf4*)q = x;
      };
      const nf4 P = ld(p + i0), Gv = ld(gr + i0), M = ld(m + i0), V = ld(v + i0);
      float pp[4] = {P.x, P.y, P.z, P.w}, gg[4] = {Gv.x, Gv.y, Gv.z, Gv.w}, mm[4] = {M.x, M.y, M.z, M.w},
            vv[4] = {V.x, V.y, V.z, V.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        mm[e] = b1 * mm[e] + (1.0f - b1) * gg[e];
        vv[e] = b2 * vv[e] + (1.0f - b2) * gg[e] * gg[e];
        const float den = sqrtf(vv[e]) * inv_sqrt_bc2 + eps;
        float np = pp[e] - ss * (mm[e] / den);
        if (clampseg) np = fminf(fmaxf(np, 0.0f), 1.0f);
        pp[e] = np;
      }
      st(p + i0, (nf4){pp[0], pp[1], pp[2], pp[3]});
      st(m + i0, (nf4){mm[0], mm[1], mm[2], mm[3]});
      st(v + i0, (nf4){vv[0], vv[1], vv[2], vv[3]});
      // a gradient float4 that is zero already is not written again (a 2^20-sample step on
      // 553.6 M parameters leaves about nine in ten untouched)
      if (Gv.x != 0.0f || Gv.y != 0.0f || Gv.z != 0.0f || Gv.w != 0.0f) st(gr + i0, (nf4){0.0f, 0.0f, 0.0f, 0.0f});
    } else {
      for (int64_t i = i0; i < n; ++i) {
        const float gg = gr[i];
        const float mm = b1 * m[i] + (1.0f - b1) * gg;
        const float vv = b2 * v[i] + (1.0f - b2) * gg * gg;
        const float den = sqrtf(vv) * inv_sqrt_bc2 + eps;
        float np = p[i] - ss * (mm / den);
        if (clampseg) np = fminf(fmaxf(np, 0.0f), 1.0f);
        p[i] = np;
        m[i] = mm;
        v[i] = vv;
        gr[i] = 0.0f;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_fill_zero(float* __restrict__ p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

// Export: one thread per (block, channel) writes the 8-byte BC4 block.
__global__ __launch_bounds__(256) void k_export_bc4(TrainDims d, const float* __restrict__ P, uint8_t* __restrict__ out) {
  const int64_t nb = (int64_t)(d.H >> 2) * (d.W >> 2) * 8;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(b & 7);
    const int64_t blk = b >> 3;
    const int bx = (int)(blk % (d.W >> 2)), by = (int)(blk / (d.W >> 2));
    const float2 e = *(const float2*)(P + b * 2);
    const int E1 = (int)rintf(__fmul_rn(255.0f, e.x)), E2 = (int)rintf(__fmul_rn(255.0f, e.y));
    uint64_t sel = 0;
    for (int s = 0; s < 16; ++s) {
      const int x = 4 * bx + (s & 3), y = 4 * by + (s >> 2);
      const int J = (int)rintf(__fmul_rn(7.0f, P[d.off_w + ((int64_t)y * d.W + x) * 8 + c]));
      int code = 0;
      if (E1 != E2) {
        const int jj = E1 > E2 ? J : 7 - J;
        code = jj == 0 ? 0 : (jj == 7 ? 1 : jj + 1);
      }
      sel |= (uint64_t)code << (3 * s);
    }
    const uint32_t e0 = (uint32_t)(E1 >= E2 ? E1 : E2), e1 = (uint32_t)(E1 >= E2 ? E2 : E1);
    const uint32_t lo = e0 | (e1 << 8) | (uint32_t)((sel & 0xffffu) << 16);
    const uint32_t hi = (uint32_t)(sel >> 16);
    *(uint2*)(out + b * 8) = make_uint2(lo, hi);
  }
}

__global__ __launch_bounds__(256) void k_convert(const float* __restrict__ src, void* __restrict__ dst, int dt, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (dt == NDGI_DTYPE_F16) ((_Float16*)dst)[i] = (_Float16)src[i];
    else ((float*)dst)[i] = src[i];
  }
}

// Tile statistics for tiled PSNR: one workgroup per tile; FP64 max, min and squared error.
__global__ __launch_bounds__(256) void k_tile_stats(const void* __restrict__ pred, int pdt,
                                                     const uint16_t* __restrict__ target, int W, int H, int tile,
                                                     double* __restrict__ stats) {
  const int tx = blockIdx.x, ty = blockIdx.y;
  const int x0 = tx * tile, y0 = ty * tile;
  const int tw = min(tile, W - x0), th = min(tile, H - y0);
  double mx = -INFINITY, mn = INFINITY, se = 0.0;
  const int64_t cnt = (int64_t)tw * th * 3;
  for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
    const int c = (int)(e % 3);
    const int64_t t = e / 3;
    const int x = x0 + (int)(t % tw), y = y0 + (int)(t / tw);
    const int64_t idx = ((int64_t)y * W + x) * 3 + c;
    const double tv = (double)half_bits(target[idx]);
    const double pv = pdt == NDGI_DTYPE_F16 ? (double)half_bits(((const uint16_t*)pred)[idx]) : (double)((const float*)pred)[idx];
    mx = fmax(mx, tv);
    mn = fmin(mn, tv);
    se += (pv - tv) * (pv - tv);
  }
  __shared__ double smx[256], smn[256], sse[256];
  smx[threadIdx.x] = mx;
  smn[threadIdx.x] = mn;
  sse[threadIdx.x] = se;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + s]);
      smn[threadIdx.x] = fmin(smn[threadIdx.x], smn[threadIdx.x + s]);
      sse[threadIdx.x] += sse[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = stats + ((size_t)ty * gridDim.x + tx) * 3;
    o[0] = smx[0];
    o[1] = smn[0];
    o[2] = sse[0];
  }
}

// Tiled PSNR from per-tile statistics [n maps][ny][nx][3] (max, min, squared error), FP64,
// one workgroup: per tile 10 log10(range^2 / MSE) over its texels and channels (range 0:
// skipped, NaN in tile_db; MSE 0: 100 dB); summary = [mean over scored tiles, global PSNR
// over every texel with the range of all tiles, least tile PSNR, scored tiles, tiles].
__global__ __launch_bounds__(256) void k_psnr(const double* __restrict__ stats, int64_t ntiles, int ny, int nx,
                                               int W, int H, int tile, double* __restrict__ tile_db,
                                               double* __restrict__ summary) {
  double sdb = 0.0, sse = 0.0, cnt = 0.0, nsc = 0.0, gmx = -INFINITY, gmn = INFINITY, dmin = INFINITY;
  for (int64_t i = threadIdx.x; i < ntiles; i += blockDim.x) {
    const int64_t r = i % ((int64_t)ny * nx);
    const int ty = (int)(r / nx), tx = (int)(r % nx);
    const double c = (double)min(tile, H - tile * ty) * (double)min(tile, W - tile * tx) * 3.0;
    const double mx = stats[3 * i], mn = stats[3 * i + 1], e = stats[3 * i + 2];
    sse += e;
    cnt += c;
    gmx = fmax(gmx, mx);
    gmn = fmin(gmn, mn);
    const double rng = mx - mn;
    double db = NAN;
    if (rng > 0.0) {
      db = e == 0.0 ? 100.0 : 10.0 * log10(rng * rng / (e / c));
      sdb += db;
      nsc += 1.0;
      dmin = fmin(dmin, db);
    }
    if (tile_db) tile_db[i] = db;
  }
  __shared__ double red[7][256];
  const double v[7] = {sdb, sse, cnt, nsc, gmx, gmn, dmin};
#pragma unroll
  for (int k = 0; k < 7; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) {
#pragma unroll
      for (int k = 0; k < 4; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
      red[4][threadIdx.x] = fmax(red[4][threadIdx.x], red[4][threadIdx.x + st]);
      red[5][threadIdx.x] = fmin(red[5][threadIdx.x], red[5][threadIdx.x + st]);
      red[6][threadIdx.x] = fmin(red[6][threadIdx.x], red[6][threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double g = red[4][0] - red[5][0];
    summary[0] = red[3][0] > 0.0 ? red[0][0] / red[3][0] : NAN;
    summary[1] = red[1][0] == 0.0 ? 100.0 : 10.0 * log10(g * g / (red[1][0] / red[2][0]));
    summary[2] = red[3][0] > 0.0 ? red[6][0] : NAN;
    summary[3] = red[3][0];
    summary[4] = (double)ntiles;
  }
}

}  // namespace ndgi

using namespace ndgi;

static int64_t param_count(int W, int H, int Gw, int Gh, int T) {
  return (int64_t)(H / 4) * (W / 4) * 16 + (int64_t)H * W * 8 + (int64_t)T * Gh * Gw * 8 + NDGI_MLP_SIZE;
}

static int check_state(const ndgi_train_state* s, const char* who) {
  if (!s) return fail(NDGI_ERR_INVALID_ARG, "%s: state is NULL", who);
  if (s->W < 4 || s->H < 4 || s->W > 4096 || s->H > 4096 || (s->W & 3) || (s->H & 3))
    return fail(NDGI_ERR_INVALID_ARG, "%s: W, H must be multiples of 4 in [4, 4096]", who);
  if (s->Gw < 1 || s->Gh < 1 || s->Gw > 4096 || s->Gh > 4096 || s->T < 1 || s->T > 256)
    return fail(NDGI_ERR_INVALID_ARG, "%s: grid %dx%d, T=%d out of range", who, s->Gw, s->Gh, s->T);
  if (!s->params || !s->grads) return fail(NDGI_ERR_INVALID_ARG, "%s: NULL params/grads", who);
  return NDGI_OK;
}

static TrainDims dims_of(const ndgi_train_state* s) {
  TrainDims d;
  d.W = s->W;
  d.H = s->H;
  d.Gw = s->Gw;
  d.Gh = s->Gh;
  d.T = s->T;
  d.off_w = (int64_t)(s->H / 4) * (s->W / 4) * 16;
  d.off_g = d.off_w + (int64_t)s->H * s->W * 8;
  d.off_mlp = d.off_g + (int64_t)s->T * s->Gh * s->Gw * 8;
  return d;
}

static int grid_for(int64_t n, int cap) {
  const int64_t w = (n + 255) / 256;
  return (int)(w < cap ? (w < 1 ? 1 : w) : cap);
}

// Host launchers of the dense kernels, shared with the hybrid-layout trainer.
namespace ndgi {
int launch_adam(ndgi_ctx* c, float* p, float* g, float* m, float* v, int64_t n, int64_t clamp_end, int64_t off_mlp,
                float lr_feat, float lr_mlp, float beta1, float beta2, float eps, int64_t step, hipStream_t s) {
  const double bc1 = 1.0 - pow((double)beta1, (double)step);
  const double bc2 = 1.0 - pow((double)beta2, (double)step);
  const float sf = (float)((double)lr_feat / bc1), sm = (float)((double)lr_mlp / bc1);
  const float isb = (float)(1.0 / sqrt(bc2));
  // streaming accesses once the state (params, grads, m, v: 16 bytes a parameter) outgrows
  // the 256 MiB last-level cache; a smaller state stays cached for the next step's gathers
  // Up to 128 workgroups a CU (about one float4 a thread at the 22 M-parameter state): the
  // stream keeps more accesses in flight than a grid-stride loop over fewer threads (a
  // 553.6 M-parameter pass took 3.68 ms at 16 a CU, 3.31 ms at 128).
  const dim3 grid(grid_for((n + 3) / 4, c->n_cu * 128));
  if (n * 16 > kLlcBytes)
    hipLaunchKernelGGL(k_adam<true>, grid, dim3(256), 0, s, p, g, m, v, n, clamp_end, off_mlp, 1.0f, 1.0f, beta1,
                       beta2, eps, sf, sm, isb);
  else
    hipLaunchKernelGGL(k_adam<false>, grid, dim3(256), 0, s, p, g, m, v, n, clamp_end, off_mlp, 1.0f, 1.0f, beta1,
                       beta2, eps, sf, sm, isb);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

int launch_fill_zero(ndgi_ctx* c, float* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(n, c->n_cu * 16)), dim3(256), 0, s, p, n);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

int launch_convert(ndgi_ctx* c, const float* src, void* dst, int dt, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_convert, dim3(grid_for(n, c->n_cu * 16)), dim3(256), 0, s, src, dst, dt, n);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}
}  // namespace ndgi

extern "C" {

int64_t ndgi_train_param_count(int32_t W, int32_t H, int32_t Gw, int32_t Gh, int32_t T) {
  return param_count(W, H, Gw, Gh, T);
}

int ndgi_train_step(ndgi_ctx* c, ndgi_train_state* st, const ndgi_batch* b, int32_t mode, double* loss_dev,
                    hipStream_t s) {
  clear_error();
  if (!c) return fail(NDGI_ERR_INVALID_ARG, "train_step: ctx is NULL");
  int rc = check_state(st, "train_step");
  if (rc) return rc;
  if (mode < NDGI_TRAIN_FORWARD || mode > NDGI_TRAIN_ZERO_GRAD) return fail(NDGI_ERR_INVALID_ARG, "train_step: bad mode %d", mode);
  const TrainDims d = dims_of(st);
  const int64_t np = d.off_mlp + NDGI_MLP_SIZE;
  if (mode == NDGI_TRAIN_ZERO_GRAD) {
    hipLaunchKernelGGL(k_fill_zero, dim3(grid_for(np, c->n_cu * 16)), dim3(256), 0, s, st->grads, np);
    NDGI_HIP(hipGetLastError());
    return NDGI_OK;
  }
  const bool needs_batch = mode != NDGI_TRAIN_ADAM;
  if (needs_batch) {
    if (!b || !b->samples || b->n < 1) return fail(NDGI_ERR_INVALID_ARG, "train_step: empty batch");
    if (mode == NDGI_TRAIN_FORWARD && !b->pred) return fail(NDGI_ERR_INVALID_ARG, "train_step: FORWARD needs pred");
    if (mode == NDGI_TRAIN_BACKWARD && !b->grad_pred)
      return fail(NDGI_ERR_INVALID_ARG, "train_step: BACKWARD needs grad_pred");
    if ((mode == NDGI_TRAIN_LOSS_GRAD || mode == NDGI_TRAIN_FUSED) && (!b->target || !loss_dev))
      return fail(NDGI_ERR_INVALID_ARG, "train_step: LOSS_GRAD/FUSED need target and loss_dev");
  }
  if ((mode == NDGI_TRAIN_ADAM || mode == NDGI_TRAIN_FUSED) && (!st->adam_m || !st->adam_v))
    return fail(NDGI_ERR_INVALID_ARG, "train_step: Adam needs adam_m, adam_v");

  if (needs_batch) {
    const int64_t groups = (b->n + 15) / 16;
    int64_t wgs = (groups + 3) / 4;
    // one round of resident workgroups, and no more waves than partial rows
    int64_t cap = resident_wgs(c, (const void*)k_train<NDGI_TRAIN_LOSS_GRAD, true>);
    if (cap > c->train_waves / 4) cap = c->train_waves / 4;
    if (wgs > cap) wgs = cap;
    const float inv3n = (float)(1.0 / (3.0 * (double)b->n));
    const bool r4 = d.W == 4 * d.Gw && d.H == 4 * d.Gh;
#define NDGI_TRAIN_LAUNCH(M)                                                                                     \
  do {                                                                                                           \
    if (r4)                                                                                                      \
      hipLaunchKernelGGL((k_train<M, true>), dim3((unsigned)wgs), dim3(256), 0, s, d, st->params, st->grads,     \
                         b->samples, b->n, b->target, b->pred, b->grad_pred, inv3n, c->partials_dev,             \
                         c->loss_part_dev, c->flags_dev);                                                        \
    else                                                                                                         \
      hipLaunchKernelGGL((k_train<M, false>), dim3((unsigned)wgs), dim3(256), 0, s, d, st->params, st->grads,    \
                         b->samples, b->n, b->target, b->pred, b->grad_pred, inv3n, c->partials_dev,             \
                         c->loss_part_dev, c->flags_dev);                                                        \
  } while (0)
    if (mode == NDGI_TRAIN_FORWARD) NDGI_TRAIN_LAUNCH(NDGI_TRAIN_FORWARD);
    else if (mode == NDGI_TRAIN_BACKWARD) NDGI_TRAIN_LAUNCH(NDGI_TRAIN_BACKWARD);
    else NDGI_TRAIN_LAUNCH(NDGI_TRAIN_LOSS_GRAD);
#undef NDGI_TRAIN_LAUNCH
    NDGI_HIP(hipGetLastError());
    if (mode != NDGI_TRAIN_FORWARD) {
      const bool want_loss = mode == NDGI_TRAIN_LOSS_GRAD || mode == NDGI_TRAIN_FUSED;
      const int rows = (int)(wgs * 4), blocks = (rows + kRowBlock - 1) / kRowBlock;
      hipLaunchKernelGGL(k_reduce_rows, dim3((NDGI_MLP_SIZE + 255) / 256, blocks), dim3(256), 0, s, c->partials_dev,
                         rows, c->stage_dev);
      hipLaunchKernelGGL(k_reduce_partials, dim3((NDGI_MLP_SIZE + 63) / 64), dim3(256), 0, s, c->stage_dev, blocks,
                         st->grads + d.off_mlp, c->loss_part_dev, rows, 1.0 / (3.0 * (double)b->n),
                         want_loss ? loss_dev : nullptr);
      NDGI_HIP(hipGetLastError());
    }
  }
  if (mode == NDGI_TRAIN_ADAM || mode == NDGI_TRAIN_FUSED) {
    const int64_t t = st->step + 1;
    rc = launch_adam(c, st->params, st->grads, st->adam_m, st->adam_v, np, d.off_g, d.off_mlp, st->lr_feat,
                     st->lr_mlp, st->beta1, st->beta2, st->eps, t, s);
    if (rc) return rc;
    st->step = t;
  }
  return NDGI_OK;
}

int ndgi_export(ndgi_ctx* c, const ndgi_train_state* st, uint8_t* bc4_out, void* grid_out, int32_t grid_dtype,
                void* mlp_out, int32_t mlp_dtype, hipStream_t s) {
  clear_error();
  if (!c) return fail(NDGI_ERR_INVALID_ARG, "export: ctx is NULL");
  int rc = check_state(st, "export");
  if (rc) return rc;
  if (!bc4_out || !grid_out || !mlp_out) return fail(NDGI_ERR_INVALID_ARG, "export: NULL output");
  if ((grid_dtype != NDGI_DTYPE_F32 && grid_dtype != NDGI_DTYPE_F16) ||
      (mlp_dtype != NDGI_DTYPE_F32 && mlp_dtype != NDGI_DTYPE_F16))
    return fail(NDGI_ERR_INVALID_ARG, "export: bad dtype");
  const TrainDims d = dims_of(st);
  const int64_t nb = (int64_t)(d.H / 4) * (d.W / 4) * 8;
  hipLaunchKernelGGL(k_export_bc4, dim3(grid_for(nb, c->n_cu * 16)), dim3(256), 0, s, d, st->params, bc4_out);
  const int64_t ng = d.off_mlp - d.off_g;
  hipLaunchKernelGGL(k_convert, dim3(grid_for(ng, c->n_cu * 16)), dim3(256), 0, s, st->params + d.off_g, grid_out,
                     grid_dtype, ng);
  hipLaunchKernelGGL(k_convert, dim3(grid_for(NDGI_MLP_SIZE, 64)), dim3(256), 0, s, st->params + d.off_mlp, mlp_out,
                     mlp_dtype, (int64_t)NDGI_MLP_SIZE);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

int ndgi_psnr(ndgi_ctx* c, const double* stats, int32_t n_maps, int32_t W, int32_t H, int32_t tile, double* tile_db,
              double* summary, hipStream_t s) {
  clear_error();
  if (!c || !stats || !summary) return fail(NDGI_ERR_INVALID_ARG, "psnr: NULL argument");
  if (n_maps < 1 || W < 1 || H < 1 || tile < 1 || tile > 4096)
    return fail(NDGI_ERR_INVALID_ARG, "psnr: bad sizes (n_maps %d, W %d, H %d, tile %d)", n_maps, W, H, tile);
  const int ny = (H + tile - 1) / tile, nx = (W + tile - 1) / tile;
  hipLaunchKernelGGL(k_psnr, dim3(1), dim3(256), 0, s, stats, (int64_t)n_maps * ny * nx, ny, nx, W, H, tile, tile_db,
                     summary);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

int ndgi_tile_stats(ndgi_ctx* c, const void* pred, int32_t pred_dtype, const uint16_t* target, int32_t W, int32_t H,
                    int32_t tile, double* stats, hipStream_t s) {
  clear_error();
  if (!c || !pred || !target || !stats) return fail(NDGI_ERR_INVALID_ARG, "tile_stats: NULL argument");
  if (W < 1 || H < 1 || tile < 1 || tile > 4096) return fail(NDGI_ERR_INVALID_ARG, "tile_stats: bad sizes");
  if (pred_dtype != NDGI_DTYPE_F32 && pred_dtype != NDGI_DTYPE_F16) return fail(NDGI_ERR_INVALID_ARG, "tile_stats: bad dtype");
  const dim3 grid((W + tile - 1) / tile, (H + tile - 1) / tile);
  hipLaunchKernelGGL(k_tile_stats, grid, dim3(256), 0, s, pred, pred_dtype, target, W, H, tile, stats);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

}  // extern "C"
