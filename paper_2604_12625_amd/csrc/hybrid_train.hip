// Training of the hybrid layout (Sec. 3.4, Eq. 6-7 and its noise equation; Sec. 4): F_uv and
// each F_uvt slice parameterised by block endpoints and per-texel weights (the paper's BC
// simulation; optionally rounded to the block format's grid) or, for the ablation, directly
// by texel values; 8-bit planes F_ut / F_vt trained in float with uniform noise standing in
// for their quantisation; the GELU decoder, L2 loss in FP64, gradients, Adam (shared with the
// other layout), export to a decodable model, and the target preprocessing (gamma,
// per-frame mean) with its inverse.
//
// One sample per lane.  A training sample is texel (x, y) of baked frame f, so its texel
// centre and frame time fix every interpolation weight.  One launch trains any number of
// models of the same sizes (the paper trains one model per virtual-texture tile): each
// model owns a contiguous run of the batch, so every workgroup's samples share one model and
// its decoder in LDS.  The decoder's forward runs in FP32 on the VALU from weights staged in
// LDS (hidden 16 or 64); its weight gradients and its input gradients run on FP32 MFMA over
// the wave's 64 samples (operands staged in LDS slabs); feature gradients go out as float
// atomics, the contended F_uvt endpoint and plane ones summed in LDS per chunk first.
#include "bcsim.hpp"
#include "hybrid.hpp"
#include "internal.hpp"

namespace ndgi {

__device__ __forceinline__ float half_bits_f(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }

// Sizes and segment offsets of one model (feature offsets relative to the model's feature
// block, F_uv endpoints first); the M models of a launch keep their feature blocks side by
// side, then their decoders: [M x o_mlp | M x (n - o_mlp)].
struct HybTrainDims {
  int W, H, Gu, Gv, S, U, V, Tt, hidden, frames;
  int M, Bm;                                          // models, samples per model
  int codec, cw;                                      // block format; weights per texel (4 or 1)
  int64_t o_uvw, o_tep, o_tw, o_ut, o_vt, o_mlp, n;   // segment offsets, parameters per model
};

static HybTrainDims htd_of(const ndgi_hybrid_train_state* st) {
  HybTrainDims d;
  d.W = st->W;
  d.H = st->H;
  d.Gu = st->Gu;
  d.Gv = st->Gv;
  d.S = st->S;
  d.U = st->U;
  d.V = st->V;
  d.Tt = st->Tt;
  d.hidden = st->hidden;
  d.frames = st->frames;
  d.M = st->n_models < 1 ? 1 : st->n_models;
  d.Bm = st->per_model;
  d.codec = st->codec;
  d.cw = d.codec == NDGI_CODEC_BC7 ? 1 : 4;
  d.o_uvw = (int64_t)(d.H / 4) * (d.W / 4) * 4 * 2;
  d.o_tep = d.o_uvw + (int64_t)d.H * d.W * d.cw;
  d.o_tw = d.o_tep + (int64_t)d.S * (d.Gv / 4) * (d.Gu / 4) * 4 * 2;
  d.o_ut = d.o_tw + (int64_t)d.S * d.Gv * d.Gu * d.cw;
  d.o_vt = d.o_ut + (int64_t)d.Tt * d.U * 2;
  d.o_mlp = d.o_vt + (int64_t)d.Tt * d.V * 2;
  d.n = d.o_mlp + ndgi_hybrid_mlp_size(d.hidden);
  return d;
}

// Counter-based uniform draw in [-1/2, 1/2): the SplitMix64 output function (Steele, Lea,
// Flood 2014) of base + counter, top 24 bits.  Exact in FP32.
__device__ __forceinline__ float hyb_noise(uint64_t base, uint64_t ctr) {
  uint64_t x = base + ctr + 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  x ^= x >> 31;
  return (float)(uint32_t)(x >> 40) * (1.0f / 16777216.0f) - 0.5f;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}


// A workgroup of 1, 2 or 4 waves takes chunks of consecutive samples of one model.  When
// the model's F_uvt endpoints and F_ut / F_vt planes fit in LDS (kAccMaxBytes), their
// gradients, the most contended ones (a footprint's endpoints collect every sample that
// taps it), are summed in LDS over the chunk and added to HBM once per chunk.
constexpr int kHtMaxThreads = 256;
constexpr int64_t kAccMaxBytes = 64 * 1024;

// The slabs are private to their wave: ordering a wave's writes before its lanes' reads is a
// wavefront-scope fence (wave_sync), and the waves of a workgroup never wait for each other
// inside a round.
// Decoder weight and bias gradients are sums over the wave's 64 samples of outer products
// of per-sample vectors, computed on MFMA with the samples as K: each operand is staged in
// an LDS slab [64 samples][16 units] (sample-major, written by the sample's lane).  Lane
// (g, i) = (lane >> 4, lane & 15) supplies sample 4 q + g, unit i of both slabs at K step q;
// the 16 x 16 result sits in lane (g, i), element r, as row 4 g + r, column i.
constexpr int kSlab = 64 * 16;
constexpr int kSlabsPerWave = 3;   // A, B, and C holding the decoder inputs during the backward

__device__ __forceinline__ void slab_store(float* slab, int lane, const float v[16]) {
  f4v* d = (f4v*)(slab + lane * 16);   // one vector type for every slab access
#pragma unroll
  for (int q = 0; q < 4; ++q) d[q] = f4v{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]};
}

// D[u][c] = acc + sum over samples of A[s][u] B[s][c]
__device__ __forceinline__ f4v slab_outer(const float* A, const float* B, int lane,
                                          f4v acc = f4v{0.0f, 0.0f, 0.0f, 0.0f}) {
  const int g = lane >> 4, i = lane & 15;
#pragma unroll
  for (int q = 0; q < 16; ++q)
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[(4 * q + g) * 16 + i], B[(4 * q + g) * 16 + i], acc, 0, 0, 0);
  return acc;
}

// D[u][c] = acc + sum over samples of A[s][u] (every column)
__device__ __forceinline__ f4v slab_sum(const float* A, int lane, f4v acc = f4v{0.0f, 0.0f, 0.0f, 0.0f}) {
  const int g = lane >> 4, i = lane & 15;
#pragma unroll
  for (int q = 0; q < 16; ++q) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A[(4 * q + g) * 16 + i], 1.0f, acc, 0, 0, 0);
  return acc;
}

// Float adds into a model's gradients in global memory, staged by the wave: lane s wrote R
// runs of L consecutive words, run r at sv[(s R + r) L ..] to words so[s R + r] + 0..L-1 of
// G (a negative offset skips the run).  An atomic add costs one memory request per 64-byte
// segment and instruction however many of the segment's words its lanes add to, so the
// 64 R L adds are issued sample-major, entry e by lane e % 64: an instruction covers the
// whole runs of 64 / (R L) samples.  Zero values are skipped (a sum that starts at +0
// never changes by adding +-0).
template <int R, int L>
__device__ __forceinline__ void ht_scatter(float* G, const float* sv, const int* so, int lane) {
  wave_sync();   // the staging is visible to the wave
#pragma unroll 1
  for (int t = 0; t < R * L; ++t) {
    const int e = 64 * t + lane;
    const int o = so[e / L];
    const float v = sv[e];
    if (o >= 0 && v != 0.0f) atomicAdd(G + o + e % L, v);
  }
  wave_sync();   // the slabs may be staged again
}

// Where a training sample reads its features: the F_uvt taps (bilinear in the grid, linear
// between slices), the F_ut / F_vt taps, and F_uv's footprint.
struct SampleTaps {
  Axis gx, gy, pu, pv;
  NodeT ns, nk;
  float tw[4];
  int txs[4], tys[4];
  int64_t fpu;
};
__device__ __forceinline__ SampleTaps sample_taps(const HybTrainDims& d, int x, int y, float tau) {
  SampleTaps T;
  T.gx = texel_axis<false>(x, d.Gu, d.W);
  T.gy = texel_axis<false>(y, d.Gv, d.H);
  T.ns = node_axis(tau, d.S);
  T.nk = node_axis(tau, d.Tt);
  tap_weights(T.gx, T.gy, T.tw);
  const int txs[4] = {T.gx.i0, T.gx.i1, T.gx.i0, T.gx.i1}, tys[4] = {T.gy.i0, T.gy.i0, T.gy.i1, T.gy.i1};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    T.txs[i] = txs[i];
    T.tys[i] = tys[i];
  }
  T.fpu = (int64_t)(y >> 2) * (d.W / 4) + (x >> 2);
  T.pu = texel_axis<false>(x, d.U, d.W);
  T.pv = texel_axis<false>(y, d.V, d.H);
  return T;
}

// MODE: NDGI_TRAIN_FORWARD writes pred; NDGI_TRAIN_LOSS_GRAD adds the loss and gradients.
// Dynamic LDS: per wave the MFMA operand slabs A, B ([64][16] each), then, with `accum`,
// the accumulators [F_uvt endpoints (nE) | F_ut, F_vt (nP)] of the chunk's model.
// `chunk` is a multiple of blockDim.x and, with several models, divides the per-model count.
template <int HD, int MODE>
__global__ __launch_bounds__(kHtMaxThreads) void k_hybrid_train(HybTrainDims d, const float* __restrict__ Pall,
                                                                 float* __restrict__ Gall,
                                                                 const float* __restrict__ keys,
                                                                 const uint32_t* __restrict__ samples, int64_t n,
                                                                 const float* __restrict__ target,
                                                                 float* __restrict__ pred, int flags,
                                                                 uint64_t noise_base, float inv3n, double loss_w,
                                                                 double* __restrict__ loss_acc, int64_t chunk,
                                                                 int accum) {
  using Sh = HybShape<HD>;
  __shared__ float sw[Sh::kSize];
  extern __shared__ __align__(16) float dyn[];   // 16-byte aligned: float4 slab accesses
  const int nthr = blockDim.x, waves = nthr >> 6;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lg = lane >> 4, li = lane & 15;
  float* const slA = dyn + wave * kSlabsPerWave * kSlab;
  float* const slB = slA + kSlab;
  float* const slC = slB + kSlab;
  float* const acc = dyn + waves * kSlabsPerWave * kSlab;
  const int64_t nE = (int64_t)d.S * (d.Gv / 4) * (d.Gu / 4) * 8, nP = d.o_mlp - d.o_ut;
  const bool bcsim = flags & NDGI_HTRAIN_BCSIM, noise = flags & NDGI_HTRAIN_NOISE, qplanes = flags & NDGI_HTRAIN_QPLANES;
  const bool direct = flags & NDGI_HTRAIN_DIRECT;
  const int64_t nchunks = (n + chunk - 1) / chunk;
  const int rounds = (int)(chunk / nthr);
  int cur = -1;
  for (int64_t ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
    const int64_t c0 = ch * chunk;
    const int m = (int)min(c0 / d.Bm, (int64_t)d.M - 1);   // the chunk lies inside one model's samples
    const float* P = Pall + (int64_t)m * d.o_mlp;
    float* G = Gall + (int64_t)m * d.o_mlp;
    const int64_t mlp_off = (int64_t)d.M * d.o_mlp + (int64_t)m * (d.n - d.o_mlp);
    float* gm = Gall + mlp_off;
    // h = 16: the decoder's weight and bias gradients of the chunk's rounds continue one MFMA
    // chain each (the next round's sums start from this round's) and reach HBM once per
    // chunk; h = 64 adds each round's (its sums would hold 85 more registers a lane)
    constexpr bool kChain = HD == 16;
    f4v cw3 = {0.0f, 0.0f, 0.0f, 0.0f}, cb3 = cw3, cw2 = cw3, cb2 = cw3, cw1 = cw3, cb1 = cw3;
  for (int r = 0; r < rounds; ++r) {
    // staging inside the round loop (first round only): the decoder weight reads of the
    // round cannot then be hoisted out of the loop into registers held across all rounds
    if (r == 0) {
      __syncthreads();   // the previous chunk's readers of sw and acc are done
      if (m != cur) {
        for (int i = threadIdx.x; i < Sh::kSize; i += nthr) sw[i] = Pall[mlp_off + i];
        cur = m;
      }
      if (accum)
        for (int64_t i = threadIdx.x; i < nE + nP; i += nthr) acc[i] = 0.0f;
      __syncthreads();
    }
    const int64_t s = c0 + (int64_t)r * nthr + threadIdx.x;
    const bool live = s < n;
    const uint32_t word = samples[live ? s : 0];
    const int x = min((int)(word & 0xfffu), d.W - 1), y = min((int)((word >> 12) & 0xfffu), d.H - 1);
    const int f = min((int)(word >> 24), d.frames - 1);
    const float tau = d.frames > 1 ? (float)f / (float)(d.frames - 1) : 0.0f;
    const float t = keys ? keys[f] : tau;
    // ---- features
    float xin[16];
    auto plane_at = [&](int64_t off, int size, int k, int a, int c) {
      const float v = P[off + ((int64_t)k * size + a) * 2 + c];
      return qplanes ? rintf(__fmul_rn(255.0f, v)) * (1.0f / 255.0f) : v;
    };
    {
    const SampleTaps T = sample_taps(d, x, y, tau);
    const NodeT &ns = T.ns, &nk = T.nk;
    const float* tw = T.tw;
    const int *txs = T.txs, *tys = T.tys;
    const int64_t fpu = T.fpu;
#pragma unroll
    for (int c = 0; c < 4; ++c) xin[c] = 0.0f;
#pragma unroll
    for (int sl = 0; sl < 2; ++sl) {
      const int si = sl ? ns.i1 : ns.i0;
      const float ws = sl ? ns.w1 : ns.w0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t fp = ((int64_t)si * (d.Gv / 4) + (tys[i] >> 2)) * (d.Gu / 4) + (txs[i] >> 2);
        const BcTex b = sim_texel(P + d.o_tep + fp * 8, P + d.o_tw + (((int64_t)si * d.Gv + tys[i]) * d.Gu + txs[i]) * d.cw,
                                  bcsim, direct, d.codec);
#pragma unroll
        for (int c = 0; c < 4; ++c) xin[c] = fmaf(ws * tw[i], b.v[c], xin[c]);
      }
    }
    {
      const BcTex bu = sim_texel(P + fpu * 8, P + d.o_uvw + ((int64_t)y * d.W + x) * d.cw, bcsim, direct, d.codec);
#pragma unroll
      for (int c = 0; c < 4; ++c) xin[4 + c] = bu.v[c];
    }
    const Axis &pu = T.pu, &pv = T.pv;
#pragma unroll
    for (int pl = 0; pl < 2; ++pl) {
      const int64_t off = pl ? d.o_vt : d.o_ut;
      const int size = pl ? d.V : d.U;
      const Axis& a = pl ? pv : pu;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        float acc = 0.0f;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
#pragma unroll
          for (int aa = 0; aa < 2; ++aa)
            acc = fmaf((kk ? nk.w1 : nk.w0) * (aa ? a.w1 : a.w0),
                       plane_at(off, size, kk ? nk.i1 : nk.i0, aa ? a.i1 : a.i0, c), acc);
        xin[8 + 2 * pl + c] = acc;
      }
    }
    }
    if (noise) {
#pragma unroll
      for (int c = 0; c < 12; ++c) xin[c] += (1.0f / 256.0f) * hyb_noise(noise_base, (uint64_t)s * 16u + (uint64_t)c);
    }
    {
      float sn, cs;
      sincospif(t, &sn, &cs);
      xin[12] = sn;
      xin[13] = cs;
      xin[14] = 2.0f * sn * cs;
      xin[15] = fmaf(cs, cs, -sn * sn);
    }
    // ---- decoder forward.  Only the layer-2 pre-activations are kept: a layer-1
    // pre-activation is recomputed (the same FMA chain) wherever it is needed again, so the
    // backward holds one 16-unit block of them at a time.
    auto pre1 = [&](int j) {
      float acc = sw[Sh::oB1 + j];
#pragma unroll
      for (int i = 0; i < 16; ++i) acc = fmaf(sw[Sh::oW1 + j * 16 + i], xin[i], acc);
      return acc;
    };
    float a2[HD];
#pragma unroll
    for (int j = 0; j < HD; ++j) a2[j] = sw[Sh::oB2 + j];
#pragma unroll
    for (int k = 0; k < HD; ++k) {
      const float h = gelu<NDGI_PREC_F32>(pre1(k));
#pragma unroll
      for (int j = 0; j < HD; ++j) a2[j] = fmaf(sw[Sh::oW2 + j * HD + k], h, a2[j]);
    }
    float out[3] = {sw[Sh::oB3], sw[Sh::oB3 + 1], sw[Sh::oB3 + 2]};
#pragma unroll
    for (int j = 0; j < HD; ++j) {
      const float h = gelu<NDGI_PREC_F32>(a2[j]);
#pragma unroll
      for (int c = 0; c < 3; ++c) out[c] = fmaf(sw[Sh::oW3 + c * HD + j], h, out[c]);
    }
    if constexpr (MODE == NDGI_TRAIN_FORWARD) {
      if (live) {
#pragma unroll
        for (int c = 0; c < 3; ++c) pred[s * 3 + c] = out[c];
      }
      continue;
    } else {
      // ---- loss and output gradient
      float dout[3];
      double sq = 0.0;
      const int64_t ti = ((((int64_t)m * d.frames + f) * d.H + y) * d.W + x) * 3;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float e = live ? out[c] - target[ti + c] : 0.0f;
        sq += (double)e * (double)e;
        dout[c] = 2.0f * inv3n * e;
      }
      sq = wave_sum_d(sq);
      if (lane == 0) atomicAdd(loss_acc, sq * loss_w);
      // ---- decoder backward.  Layer 3: dW3[c][j] = sum dout[c] h2[j], db3 = sum dout
      {
        float v[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = c < 3 ? dout[c] : 0.0f;
        slab_store(slA, lane, v);
      }
#pragma unroll
      for (int jb = 0; jb < HD / 16; ++jb) {
        float v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) v[u] = gelu<NDGI_PREC_F32>(a2[16 * jb + u]);
        slab_store(slB, lane, v);
        wave_sync();
        if constexpr (kChain) {
          cw3 = slab_outer(slA, slB, lane, cw3);
          cb3 = slab_sum(slA, lane, cb3);
        } else {
          const f4v w3 = slab_outer(slA, slB, lane);
          if (lg == 0) {
#pragma unroll
            for (int r = 0; r < 3; ++r) atomicAdd(gm + Sh::oW3 + r * HD + 16 * jb + li, w3[r]);
          }
          if (jb == 0) {
            const f4v b3 = slab_sum(slA, lane);
            if (lane == 0) {
#pragma unroll
              for (int r = 0; r < 3; ++r) atomicAdd(gm + Sh::oB3 + r, b3[r]);
            }
          }
        }
        wave_sync();
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int j = 0; j < HD; ++j) {
        float dh = 0.0f;
#pragma unroll
        for (int c = 0; c < 3; ++c) dh = fmaf(sw[Sh::oW3 + c * HD + j], dout[c], dh);
        a2[j] = dh * gelu_grad(a2[j]);   // a2 now holds d loss / d a2
      }
      // Layers 2 and 1, one 16-unit block kb of layer 1 at a time.  Layer 2: dW2[j][k] =
      // sum g2[j] h1[k], db2 = sum g2 (g2 = d loss / d a2); the input gradient DH[k][s] =
      // sum_j W2[j][k] g2[s][j] on MFMA as well (W2 from LDS as the A operand, the staged g2
      // slab as B), handed back to the sample lanes through LDS, giving the block's
      // g1 = DH gelu'(a1).  Layer 1 for that block: dW1[k][i] = sum g1[k] x[i], db1 = sum g1,
      // and its share of the input gradient DX[i][s] = sum_k W1[k][i] g1[s][k], on MFMA.
      slab_store(slC, lane, xin);
      // the decoder inputs are read back from the lane's own row of slab C (written by this
      // lane, so no barrier) rather than kept in registers through the backward
      auto pre1c = [&](int j) {
        const f4v* xr = (const f4v*)(slC + lane * 16);
        float acc = sw[Sh::oB1 + j];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const f4v xq = xr[q];
#pragma unroll
          for (int e = 0; e < 4; ++e) acc = fmaf(sw[Sh::oW1 + j * 16 + 4 * q + e], xq[e], acc);
        }
        return acc;
      };
      f4v dx4[4];
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) dx4[sb] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
      for (int kb = 0; kb < HD / 16; ++kb) {
        float a1b[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) a1b[u] = pre1c(16 * kb + u);
        {
          float v[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) v[u] = gelu<NDGI_PREC_F32>(a1b[u]);
          slab_store(slB, lane, v);
        }
        f4v dh4[4];
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) dh4[sb] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int jb = 0; jb < HD / 16; ++jb) {
          slab_store(slA, lane, a2 + 16 * jb);
          wave_sync();
          if constexpr (kChain) {
            cw2 = slab_outer(slA, slB, lane, cw2);
            cb2 = slab_sum(slA, lane, cb2);
          } else {
            const f4v w2 = slab_outer(slA, slB, lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) atomicAdd(gm + Sh::oW2 + (16 * jb + 4 * lg + r) * HD + 16 * kb + li, w2[r]);
            if (kb == 0) {
              const f4v b2 = slab_sum(slA, lane);
              if (li == 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) atomicAdd(gm + Sh::oB2 + 16 * jb + 4 * lg + r, b2[r]);
              }
            }
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const float wa = sw[Sh::oW2 + (16 * jb + 4 * q + lg) * HD + 16 * kb + li];
#pragma unroll
            for (int sb = 0; sb < 4; ++sb)
              dh4[sb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa, slA[(16 * sb + li) * 16 + 4 * q + lg], dh4[sb], 0, 0,
                                                             0);
          }
          wave_sync();
          __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int sb = 0; sb < 4; ++sb) *(f4v*)(slB + (16 * sb + li) * 16 + 4 * lg) = dh4[sb];
        wave_sync();
        {
          const f4v* own = (const f4v*)(slB + lane * 16);
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const f4v dq = own[q];
#pragma unroll
            for (int e = 0; e < 4; ++e) a1b[4 * q + e] = dq[e] * gelu_grad(a1b[4 * q + e]);   // now g1
          }
        }
        slab_store(slA, lane, a1b);
        wave_sync();
        if constexpr (kChain) {
          cw1 = slab_outer(slA, slC, lane, cw1);
          cb1 = slab_sum(slA, lane, cb1);
        } else {
          const f4v w1 = slab_outer(slA, slC, lane);
#pragma unroll
          for (int r = 0; r < 4; ++r) atomicAdd(gm + Sh::oW1 + (16 * kb + 4 * lg + r) * 16 + li, w1[r]);
          const f4v b1 = slab_sum(slA, lane);
          if (li == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) atomicAdd(gm + Sh::oB1 + 16 * kb + 4 * lg + r, b1[r]);
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float wa = sw[Sh::oW1 + (16 * kb + 4 * q + lg) * 16 + li];
#pragma unroll
          for (int sb = 0; sb < 4; ++sb)
            dx4[sb] = __builtin_amdgcn_mfma_f32_16x16x4f32(wa, slA[(16 * sb + li) * 16 + 4 * q + lg], dx4[sb], 0, 0, 0);
        }
        wave_sync();
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int sb = 0; sb < 4; ++sb) *(f4v*)(slB + (16 * sb + li) * 16 + 4 * lg) = dx4[sb];
      wave_sync();
      float dx[16];
      {
        const f4v* own = (const f4v*)(slB + lane * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const f4v dq = own[q];
#pragma unroll
          for (int e = 0; e < 4; ++e) dx[4 * q + e] = dq[e];
        }
      }
      wave_sync();   // every lane holds its dx: the slabs take the scatter staging below
      // The taps again, recomputed from the sample's texel and time rather than kept through
      // the decoder backward (the empty asm hides that they equal the forward's, so they are
      // not reused from it).
      int xr = x, yr = y;
      float taur = tau;
      asm volatile("" : "+v"(xr), "+v"(yr), "+v"(taur));
      const SampleTaps T = sample_taps(d, xr, yr, taur);
      const NodeT &ns = T.ns, &nk = T.nk;
      const float* tw = T.tw;
      const int *txs = T.txs, *tys = T.tys;
      const int64_t fpu = T.fpu;
      const Axis &pu = T.pu, &pv = T.pv;
      // ---- feature gradients (straight-through for the simulated maps).  Adds into HBM go
      // through the wave's slabs in runs of consecutive words (ht_scatter), so that an
      // instruction covers whole runs of a few samples; adds into the chunk's LDS
      // accumulators are issued per lane.  Dead lanes stage skipped runs.
      float* const sv = slA;          // staged values [64][R x L] (slabs A and B)
      int* const so = (int*)slC;      // staged run offsets into G [64][R]; negative skips
      // Per F_uvt slice the four taps' endpoint terms are first summed per 4x4 footprint (taps
      // 0/1 and 2/3 share one when their columns do, taps 0/2 and 1/3 when their rows do), so
      // each footprint the sample touches takes one set of 8 adds.
      const bool fsx = (txs[0] >> 2) == (txs[1] >> 2), fsy = (tys[0] >> 2) == (tys[2] >> 2);
#pragma unroll
      for (int sl = 0; sl < 2; ++sl) {
        const int si = sl ? ns.i1 : ns.i0;
        const float ws = sl ? ns.w1 : ns.w0;
        float e[4][8];
        int64_t fps[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t fp = ((int64_t)si * (d.Gv / 4) + (tys[i] >> 2)) * (d.Gu / 4) + (txs[i] >> 2);
          const int64_t wi = (((int64_t)si * d.Gv + tys[i]) * d.Gu + txs[i]) * d.cw;
          const BcTex b = sim_texel(P + d.o_tep + fp * 8, P + d.o_tw + wi, bcsim, direct, d.codec);
          const float wt = ws * tw[i];
          fps[i] = fp;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const float dv = wt * dx[c];
            e[i][2 * c] = dv * b.d1[c];
            e[i][2 * c + 1] = dv * b.d2[c];
            if (!d.codec) sv[lane * 16 + 4 * i + c] = dv * b.dw[c];
          }
          if (d.codec) sv[lane * 4 + i] = wt * (dx[0] * b.dw[0] + dx[1] * b.dw[1] + dx[2] * b.dw[2] + dx[3] * b.dw[3]);
          so[lane * 4 + i] = live ? (int)(d.o_tw + wi) : -1;
        }
        if (d.codec) ht_scatter<4, 1>(G, sv, so, lane);
        else ht_scatter<4, 4>(G, sv, so, lane);
        if (direct) continue;   // a directly optimised map has no endpoints
        if (fsx) {
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            e[0][k] += e[1][k];
            e[2][k] += e[3][k];
          }
        }
        if (fsy) {
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            e[0][k] += e[2][k];
            e[1][k] += e[3][k];   // unused when fsx (tap 1 then merged into tap 0 already)
          }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const bool own = live && (i == 0 || (i == 1 && !fsx) || (i == 2 && !fsy) || (i == 3 && !fsx && !fsy));
          if (accum) {
            if (own) {
#pragma unroll
              for (int k = 0; k < 8; ++k) atomicAdd(acc + fps[i] * 8 + k, e[i][k]);   // LDS (ds_add)
            }
          } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) sv[lane * 32 + 8 * i + k] = e[i][k];
            so[lane * 4 + i] = own ? (int)(d.o_tep + fps[i] * 8) : -1;
          }
        }
        if (!accum) ht_scatter<4, 8>(G, sv, so, lane);
      }
      // F_uv's texel again (recomputed rather than kept through the decoder backward)
      const BcTex bu = sim_texel(P + fpu * 8, P + d.o_uvw + ((int64_t)y * d.W + x) * d.cw, bcsim, direct, d.codec);
      if (!direct) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          sv[lane * 8 + 2 * c] = dx[4 + c] * bu.d1[c];
          sv[lane * 8 + 2 * c + 1] = dx[4 + c] * bu.d2[c];
        }
        so[lane] = live ? (int)(fpu * 8) : -1;
        ht_scatter<1, 8>(G, sv, so, lane);
      }
      if (!d.codec) {
#pragma unroll
        for (int c = 0; c < 4; ++c) sv[lane * 4 + c] = dx[4 + c] * bu.dw[c];
        so[lane] = live ? (int)(d.o_uvw + ((int64_t)y * d.W + x) * 4) : -1;
        ht_scatter<1, 4>(G, sv, so, lane);
      } else if (live) {
        atomicAdd(G + d.o_uvw + (int64_t)y * d.W + x,
                  dx[4] * bu.dw[0] + dx[5] * bu.dw[1] + dx[6] * bu.dw[2] + dx[7] * bu.dw[3]);
      }
#pragma unroll
      for (int pl = 0; pl < 2; ++pl) {
        const int64_t off = pl ? d.o_vt : d.o_ut;
        const int size = pl ? d.V : d.U;
        const Axis& a = pl ? pv : pu;
#pragma unroll
        for (int kk = 0; kk < 2; ++kk)
#pragma unroll
          for (int aa = 0; aa < 2; ++aa) {
            const float w = (kk ? nk.w1 : nk.w0) * (aa ? a.w1 : a.w0);
            const int64_t idx = off + ((int64_t)(kk ? nk.i1 : nk.i0) * size + (aa ? a.i1 : a.i0)) * 2;
            const int tap = 4 * pl + 2 * kk + aa;
            if (accum) {
              if (live) {
                atomicAdd(acc + nE + (idx - d.o_ut), w * dx[8 + 2 * pl]);
                atomicAdd(acc + nE + (idx - d.o_ut) + 1, w * dx[9 + 2 * pl]);
              }
            } else {
              sv[lane * 16 + 2 * tap] = w * dx[8 + 2 * pl];
              sv[lane * 16 + 2 * tap + 1] = w * dx[9 + 2 * pl];
              so[lane * 8 + tap] = live ? (int)idx : -1;
            }
          }
      }
      if (!accum) ht_scatter<8, 2>(G, sv, so, lane);
    }
  }
    if constexpr (kChain && MODE != NDGI_TRAIN_FORWARD) {   // the chunk's decoder sums into HBM
      if (lg == 0) {
#pragma unroll
        for (int r = 0; r < 3; ++r) atomicAdd(gm + Sh::oW3 + r * HD + li, cw3[r]);
      }
      if (lane == 0) {
#pragma unroll
        for (int r = 0; r < 3; ++r) atomicAdd(gm + Sh::oB3 + r, cb3[r]);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        atomicAdd(gm + Sh::oW2 + (4 * lg + r) * HD + li, cw2[r]);
        atomicAdd(gm + Sh::oW1 + (4 * lg + r) * 16 + li, cw1[r]);
      }
      if (li == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          atomicAdd(gm + Sh::oB2 + 4 * lg + r, cb2[r]);
          atomicAdd(gm + Sh::oB1 + 4 * lg + r, cb1[r]);
        }
      }
    }
    if (accum) {   // the chunk's sums into HBM
      __syncthreads();
      for (int64_t i = threadIdx.x; i < nE; i += nthr) {
        const float v = acc[i];
        if (v != 0.0f) atomicAdd(G + d.o_tep + i, v);
      }
      for (int64_t i = threadIdx.x; i < nP; i += nthr) {
        const float v = acc[nE + i];
        if (v != 0.0f) atomicAdd(G + d.o_ut + i, v);
      }
    }
  }
}

__global__ void k_zero_d(double* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0.0;
}

// Export of a C-channel BC-simulated map ([H/4][W/4][C][2] endpoints, [H][W][C] weights) to
// BC4 blocks [H/4][W/4][C][8], the encoding of the other layout's export.
__global__ __launch_bounds__(256) void k_export_bc4c(const float* __restrict__ ep, const float* __restrict__ wts, int W,
                                                      int H, int C, int64_t nb, uint8_t* __restrict__ out) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(b % C);
    const int64_t blk = b / C;
    const int64_t per = (int64_t)(H >> 2) * (W >> 2);
    const int64_t sl = blk / per, rem = blk - sl * per;
    const int bx = (int)(rem % (W >> 2)), by = (int)(rem / (W >> 2));
    const float2 e = *(const float2*)(ep + b * 2);
    const int E1 = (int)rintf(__fmul_rn(255.0f, e.x)), E2 = (int)rintf(__fmul_rn(255.0f, e.y));
    uint64_t sel = 0;
    for (int s = 0; s < 16; ++s) {
      const int x = 4 * bx + (s & 3), y = 4 * by + (s >> 2);
      const int J = (int)rintf(__fmul_rn(7.0f, wts[((sl * H + y) * W + x) * C + c]));
      int code = 0;
      if (E1 != E2) {
        const int jj = E1 > E2 ? J : 7 - J;
        code = jj == 0 ? 0 : (jj == 7 ? 1 : jj + 1);
      }
      sel |= (uint64_t)code << (3 * s);
    }
    const uint32_t e0 = (uint32_t)(E1 >= E2 ? E1 : E2), e1 = (uint32_t)(E1 >= E2 ? E2 : E1);
    *(uint2*)(out + b * 8) = make_uint2(e0 | (e1 << 8) | (uint32_t)((sel & 0xffffu) << 16), (uint32_t)(sel >> 16));
  }
}

// Export of a BC7-simulated 4-channel map ([..][H/4][W/4][4][2] endpoints, [..][H][W] weights)
// to mode-6 blocks [..][H/4][W/4][16]: endpoints as in the simulation, J = rint(fl32(15 w));
// when texel 0's index has its top bit set the endpoints swap and every index becomes
// 15 - J (the weight table is symmetric), so the decode equals the simulation.
__global__ __launch_bounds__(256) void k_export_bc7(const float* __restrict__ ep, const float* __restrict__ wts, int W,
                                                     int H, int64_t nb, uint8_t* __restrict__ out) {
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nb; b += (int64_t)gridDim.x * blockDim.x) {
    const int64_t per = (int64_t)(H >> 2) * (W >> 2);
    const int64_t sl = b / per, rem = b - sl * per;
    const int bx = (int)(rem % (W >> 2)), by = (int)(rem / (W >> 2));
    const float4 ea = *(const float4*)(ep + b * 8), eb = *(const float4*)(ep + b * 8 + 4);
    const float e1[4] = {ea.x, ea.z, eb.x, eb.z}, e2[4] = {ea.y, ea.w, eb.y, eb.w};
    int E[2][4];
    bc7_endpoint(e1, E[0]);
    bc7_endpoint(e2, E[1]);
    int J[16];
    for (int s = 0; s < 16; ++s) {
      const int x = 4 * bx + (s & 3), y = 4 * by + (s >> 2);
      J[s] = (int)rintf(__fmul_rn(15.0f, wts[(sl * H + y) * W + x]));
    }
    const bool swap = J[0] >= 8;
    uint64_t lo = 0x40, hi = 0;
    for (int c = 0; c < 4; ++c) {
      const int a = E[swap ? 1 : 0][c], z = E[swap ? 0 : 1][c];
      lo |= (uint64_t)(a >> 1) << (7 + 14 * c);
      lo |= (uint64_t)(z >> 1) << (14 + 14 * c);
    }
    lo |= (uint64_t)(E[swap ? 1 : 0][0] & 1) << 63;
    hi |= (uint64_t)(E[swap ? 0 : 1][0] & 1);
    for (int s = 0; s < 16; ++s) {
      const uint64_t j = (uint64_t)(swap ? 15 - J[s] : J[s]);
      hi |= s ? j << (4 * s) : j << 1;
    }
    *(u4v*)(out + b * 16) = (u4v){(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32)};
  }
}

// 8-bit planes: q = rint(fl32(255 v)) of values already projected to [0, 1].
__global__ __launch_bounds__(256) void k_quant8(const float* __restrict__ src, uint8_t* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (uint8_t)min(max((int)rintf(__fmul_rn(255.0f, src[i])), 0), 255);
}

// Import helpers: block endpoints (e1, e2) = (0, 1), so that the Eq. 7 lerp reads the weight
// itself; 8-bit planes as byte / 255; a decoder of either dtype as float.
__global__ __launch_bounds__(256) void k_fill_ep01(float* __restrict__ ep, int64_t pairs) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < pairs; i += (int64_t)gridDim.x * blockDim.x)
    *(float2*)(ep + 2 * i) = make_float2(0.0f, 1.0f);
}

__global__ __launch_bounds__(256) void k_unit8(const uint8_t* __restrict__ src, float* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i] / 255.0f;
}

__global__ __launch_bounds__(256) void k_to_f32(const void* __restrict__ src, int dt, float* __restrict__ dst,
                                                 int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = dt == NDGI_DTYPE_F16 ? (float)((const _Float16*)src)[i] : ((const float*)src)[i];
}

// Target preprocessing (Sec. 4): y^(1/gamma) per texel and channel; per frame and channel the
// FP64 sum, then division by the mean.  One workgroup per (frame, 64K-texel chunk).
constexpr int kNormChunk = 65536;
__global__ __launch_bounds__(256) void k_norm_sum(const uint16_t* __restrict__ tgt, int64_t texels, float inv_gamma,
                                                   double* __restrict__ sums) {
  const int f = blockIdx.y;
  const int64_t lo = (int64_t)blockIdx.x * kNormChunk, hi = min(texels, lo + kNormChunk);
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      acc[c] += (double)powf(half_bits_f(tgt[((int64_t)f * texels + i) * 3 + c]), inv_gamma);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double v = wave_sum_d(acc[c]);
    if ((threadIdx.x & 63) == 0) atomicAdd(sums + f * 3 + c, v);
  }
}

__global__ __launch_bounds__(256) void k_norm_apply(const uint16_t* __restrict__ tgt, int64_t texels, int frames,
                                                     float inv_gamma, double* __restrict__ sums,
                                                     float* __restrict__ out) {
  const int64_t total = (int64_t)frames * texels * 3;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t f = i / (texels * 3);
    const int c = (int)(i % 3);
    const double mean = sums[f * 3 + c] / (double)texels;
    out[i] = (float)((double)powf(half_bits_f(tgt[i]), inv_gamma) / mean);
  }
}

__global__ void k_norm_means(double* sums, int n, int64_t texels) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) sums[i] /= (double)texels;
}

// Inverse for one decoded frame: max(pred * mean, 0)^gamma.
__global__ __launch_bounds__(256) void k_restore(const void* __restrict__ pred, int pdt, int64_t texels,
                                                  const double* __restrict__ mean3, float gamma, float* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < texels * 3; i += (int64_t)gridDim.x * blockDim.x) {
    const float p = pdt == NDGI_DTYPE_F16 ? (float)((const _Float16*)pred)[i] : ((const float*)pred)[i];
    const float v = p * (float)mean3[i % 3];
    out[i] = v > 0.0f ? powf(v, gamma) : 0.0f;
  }
}

static int grid_of(int64_t n, int cap) {
  const int64_t w = (n + 255) / 256;
  return (int)(w < cap ? (w < 1 ? 1 : w) : cap);
}

static int check_htrain(const ndgi_hybrid_train_state* st, const char* who) {
  if (!st) return fail(NDGI_ERR_INVALID_ARG, "%s: state is NULL", who);
  ndgi_hybrid_model m = {};
  m.W = st->W;
  m.H = st->H;
  m.Gu = st->Gu;
  m.Gv = st->Gv;
  m.S = st->S;
  m.U = st->U;
  m.V = st->V;
  m.Tt = st->Tt;
  m.hidden = st->hidden;
  m.mlp_dtype = NDGI_DTYPE_F32;
  m.codec = st->codec;
  m.fuv = m.fuvt = m.fut = m.fvt = (const uint8_t*)st->params;
  m.mlp = st->params;
  if (!st->params || !st->grads) return fail(NDGI_ERR_INVALID_ARG, "%s: NULL params/grads", who);
  int rc = check_hybrid(&m, who);
  if (rc) return rc;
  if (st->W > 4096 || st->H > 4096) return fail(NDGI_ERR_INVALID_ARG, "%s: W, H above 4096", who);
  if (st->frames < 1 || st->frames > 256) return fail(NDGI_ERR_INVALID_ARG, "%s: frames=%d not in 1..256", who, st->frames);
  if (st->n_models < 1) return fail(NDGI_ERR_INVALID_ARG, "%s: n_models=%d < 1", who, st->n_models);
  if (st->n_models > 1 && ((int64_t)st->Tt * (st->U + st->V)) % 2)
    return fail(NDGI_ERR_INVALID_ARG, "%s: with several models Tt * (U + V) must be even (16-byte aligned model blocks)",
                who);
  if (st->reserved0) return fail(NDGI_ERR_INVALID_ARG, "%s: reserved0 must be 0", who);
  if (htd_of(st).o_mlp > INT32_MAX)   // the gradient scatter stages 32-bit offsets
    return fail(NDGI_ERR_INVALID_ARG, "%s: a model's feature block exceeds 2^31 words", who);
  return NDGI_OK;
}

}  // namespace ndgi

using namespace ndgi;

extern "C" {

int64_t ndgi_hybrid_train_param_count(int32_t W, int32_t H, int32_t Gu, int32_t Gv, int32_t S, int32_t U, int32_t V,
                                      int32_t Tt, int32_t hidden, int32_t codec) {
  if (ndgi_hybrid_mlp_size(hidden) < 0 || W < 4 || H < 4 || Gu < 4 || Gv < 4 || S < 1 || U < 1 || V < 1 || Tt < 1 ||
      (codec != NDGI_CODEC_BC4 && codec != NDGI_CODEC_BC7))
    return -1;
  ndgi_hybrid_train_state st = {};
  st.W = W;
  st.H = H;
  st.Gu = Gu;
  st.Gv = Gv;
  st.S = S;
  st.U = U;
  st.V = V;
  st.Tt = Tt;
  st.hidden = hidden;
  st.codec = codec;
  st.frames = 1;
  return htd_of(&st).n;
}

int ndgi_hybrid_train_step(ndgi_ctx* c, ndgi_hybrid_train_state* st, const ndgi_hybrid_batch* b, int32_t mode,
                           int32_t flags, double* loss_dev, hipStream_t s) {
  clear_error();
  if (!c) return fail(NDGI_ERR_INVALID_ARG, "hybrid_train_step: ctx is NULL");
  int rc = check_htrain(st, "hybrid_train_step");
  if (rc) return rc;
  if (mode != NDGI_TRAIN_FORWARD && mode != NDGI_TRAIN_LOSS_GRAD && mode != NDGI_TRAIN_FUSED &&
      mode != NDGI_TRAIN_ADAM && mode != NDGI_TRAIN_ZERO_GRAD)
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_train_step: unsupported mode %d", mode);
  if (flags & ~(NDGI_HTRAIN_BCSIM | NDGI_HTRAIN_NOISE | NDGI_HTRAIN_QPLANES | NDGI_HTRAIN_DIRECT))
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_train_step: unknown flags 0x%x", flags);
  if ((flags & NDGI_HTRAIN_DIRECT) && ((flags & NDGI_HTRAIN_BCSIM) || st->codec != NDGI_CODEC_BC4))
    return fail(NDGI_ERR_INVALID_ARG,
                "hybrid_train_step: DIRECT needs a state in the BC4 layout (one value per texel and channel) and "
                "excludes BCSIM");
  const HybTrainDims d = htd_of(st);
  const int64_t total = (int64_t)d.M * d.n;
  if (mode == NDGI_TRAIN_ZERO_GRAD) return launch_fill_zero(c, st->grads, total, s);
  const bool needs_batch = mode != NDGI_TRAIN_ADAM;
  if (needs_batch) {
    if (!b || !b->samples || b->n < 1 || b->n > INT32_MAX)
      return fail(NDGI_ERR_INVALID_ARG, "hybrid_train_step: batch of 1..2^31-1 samples needed");
    if (mode == NDGI_TRAIN_FORWARD && !b->pred) return fail(NDGI_ERR_INVALID_ARG, "hybrid_train_step: FORWARD needs pred");
    if (mode != NDGI_TRAIN_FORWARD && (!b->target || !loss_dev))
      return fail(NDGI_ERR_INVALID_ARG, "hybrid_train_step: LOSS_GRAD/FUSED need target and loss_dev");
    if (d.M > 1 && (d.Bm < 64 || d.Bm % 64 || (int64_t)d.Bm * d.M != b->n))
      return fail(NDGI_ERR_INVALID_ARG,
                  "hybrid_train_step: %d models need per_model a multiple of 64 with n = n_models * per_model", d.M);
  }
  if ((mode == NDGI_TRAIN_ADAM || mode == NDGI_TRAIN_FUSED) && (!st->adam_m || !st->adam_v))
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_train_step: Adam needs adam_m, adam_v");
  if (needs_batch) {
    HybTrainDims dl = d;
    if (dl.M == 1) dl.Bm = (int)b->n;
    const uint64_t base = (uint64_t)st->seed * 0x9E3779B97F4A7C15ull + ((uint64_t)st->step << 32);
    // each model's loss is the mean over its own samples; the launch reports the mean of the
    // models' losses
    const float inv3n = (float)(1.0 / (3.0 * (double)dl.Bm));
    const double loss_w = 1.0 / (3.0 * (double)dl.Bm * (double)dl.M);
    // workgroup size: one wave for small batches (spread over the CUs), else 4 waves (2 or 1
    // when a model's sample count is not a multiple of 256); chunks of k workgroup rounds,
    // k up to 16 while the grid keeps about one chunk per CU
    int nthr = b->n >= (int64_t)64 * c->n_cu ? kHtMaxThreads : 64;
    if (dl.M > 1)
      while (nthr > 64 && dl.Bm % nthr != 0) nthr >>= 1;
    int64_t k = b->n / ((int64_t)nthr * c->n_cu);
    k = k < 1 ? 1 : (k > 16 ? 16 : k);
    while (k > 1 && dl.M > 1 && dl.Bm % (nthr * k) != 0) --k;
    const int64_t chunk = (int64_t)nthr * k;
    int64_t wgs = (b->n + chunk - 1) / chunk;
    const int64_t cap = (int64_t)c->n_cu * 8;
    if (wgs > cap) wgs = cap;
    const int64_t nE = (int64_t)d.S * (d.Gv / 4) * (d.Gu / 4) * 8, nP = d.o_mlp - d.o_ut;
    const size_t slab_bytes = (size_t)(nthr / 64) * kSlabsPerWave * kSlab * sizeof(float);
    const size_t acc_bytes = (size_t)(nE + nP) * sizeof(float);
    const size_t sw_bytes = ((size_t)ndgi_hybrid_mlp_size(d.hidden) * sizeof(float) + 15) / 16 * 16;   // static LDS
    int lds_max = 0;
    NDGI_HIP(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
    // LDS sums pay off when a chunk has several waves' samples or models share the launch
    const int accum = mode != NDGI_TRAIN_FORWARD && (nthr > 64 || dl.M > 1) && (int64_t)acc_bytes <= kAccMaxBytes &&
                      sw_bytes + slab_bytes + acc_bytes <= (size_t)lds_max;
    const size_t dyn_bytes = slab_bytes + (accum ? acc_bytes : 0);
    if (mode != NDGI_TRAIN_FORWARD) hipLaunchKernelGGL(k_zero_d, dim3(1), dim3(64), 0, s, loss_dev, 1);
#define NDGI_HT(HD, M)                                                                                          \
  hipLaunchKernelGGL((k_hybrid_train<HD, M>), dim3((unsigned)wgs), dim3(nthr), dyn_bytes, s, dl, st->params,      \
                     st->grads, st->keys, b->samples, b->n, b->target, b->pred, flags, base, inv3n, loss_w, loss_dev, chunk, \
                     accum)
    if (mode == NDGI_TRAIN_FORWARD) {
      if (d.hidden == 16) NDGI_HT(16, NDGI_TRAIN_FORWARD);
      else NDGI_HT(64, NDGI_TRAIN_FORWARD);
    } else {
      if (d.hidden == 16) NDGI_HT(16, NDGI_TRAIN_LOSS_GRAD);
      else NDGI_HT(64, NDGI_TRAIN_LOSS_GRAD);
    }
#undef NDGI_HT
    NDGI_HIP(hipGetLastError());
  }
  if (mode == NDGI_TRAIN_ADAM || mode == NDGI_TRAIN_FUSED) {
    // every feature map is projected to [0, 1]; the decoder is not
    rc = launch_adam(c, st->params, st->grads, st->adam_m, st->adam_v, total, (int64_t)d.M * d.o_mlp,
                     (int64_t)d.M * d.o_mlp, st->lr_feat,
                     st->lr_mlp, st->beta1, st->beta2, st->eps, st->step + 1, s);
    if (rc) return rc;
    st->step += 1;
  }
  return NDGI_OK;
}

int ndgi_hybrid_export(ndgi_ctx* c, const ndgi_hybrid_train_state* st, int32_t model, uint8_t* fuv_out,
                       uint8_t* fuvt_out, uint8_t* fut_out, uint8_t* fvt_out, void* mlp_out, int32_t mlp_dtype,
                       hipStream_t s) {
  clear_error();
  if (!c) return fail(NDGI_ERR_INVALID_ARG, "hybrid_export: ctx is NULL");
  int rc = check_htrain(st, "hybrid_export");
  if (rc) return rc;
  if (!fuv_out || !fuvt_out || !fut_out || !fvt_out || !mlp_out)
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_export: NULL output");
  if (mlp_dtype != NDGI_DTYPE_F32 && mlp_dtype != NDGI_DTYPE_F16)
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_export: bad dtype");
  const HybTrainDims d = htd_of(st);
  if (model < 0 || model >= d.M) return fail(NDGI_ERR_INVALID_ARG, "hybrid_export: model %d of %d", model, d.M);
  const float* P = st->params + (int64_t)model * d.o_mlp;
  const float* mlp = st->params + (int64_t)d.M * d.o_mlp + (int64_t)model * (d.n - d.o_mlp);
  const int64_t nb_uv = (int64_t)(d.H / 4) * (d.W / 4) * 4, nb_uvt = (int64_t)d.S * (d.Gv / 4) * (d.Gu / 4) * 4;
  if (d.codec == NDGI_CODEC_BC7) {
    const int64_t fb_uv = nb_uv / 4, fb_uvt = nb_uvt / 4;   // footprints
    hipLaunchKernelGGL(k_export_bc7, dim3(grid_of(fb_uv, c->n_cu * 16)), dim3(256), 0, s, P, P + d.o_uvw, d.W, d.H,
                       fb_uv, fuv_out);
    hipLaunchKernelGGL(k_export_bc7, dim3(grid_of(fb_uvt, c->n_cu * 16)), dim3(256), 0, s, P + d.o_tep, P + d.o_tw,
                       d.Gu, d.Gv, fb_uvt, fuvt_out);
  } else {
    hipLaunchKernelGGL(k_export_bc4c, dim3(grid_of(nb_uv, c->n_cu * 16)), dim3(256), 0, s, P, P + d.o_uvw, d.W,
                       d.H, 4, nb_uv, fuv_out);
    hipLaunchKernelGGL(k_export_bc4c, dim3(grid_of(nb_uvt, c->n_cu * 16)), dim3(256), 0, s, P + d.o_tep,
                       P + d.o_tw, d.Gu, d.Gv, 4, nb_uvt, fuvt_out);
  }
  hipLaunchKernelGGL(k_quant8, dim3(grid_of((int64_t)d.Tt * d.U * 2, 1024)), dim3(256), 0, s, P + d.o_ut, fut_out,
                     (int64_t)d.Tt * d.U * 2);
  hipLaunchKernelGGL(k_quant8, dim3(grid_of((int64_t)d.Tt * d.V * 2, 1024)), dim3(256), 0, s, P + d.o_vt, fvt_out,
                     (int64_t)d.Tt * d.V * 2);
  NDGI_HIP(hipGetLastError());
  return launch_convert(c, mlp, mlp_out, mlp_dtype, d.n - d.o_mlp, s);
}

int ndgi_hybrid_encode(ndgi_ctx* c, const ndgi_hybrid_train_state* st, int32_t model, int32_t flags, int32_t codec,
                       uint8_t* fuv_out, uint8_t* fuvt_out, uint8_t* fut_out, uint8_t* fvt_out, void* mlp_out,
                       int32_t mlp_dtype, hipStream_t s) {
  clear_error();
  if (!c) return fail(NDGI_ERR_INVALID_ARG, "hybrid_encode: ctx is NULL");
  int rc = check_htrain(st, "hybrid_encode");
  if (rc) return rc;
  if (flags & ~(NDGI_HTRAIN_BCSIM | NDGI_HTRAIN_NOISE | NDGI_HTRAIN_QPLANES | NDGI_HTRAIN_DIRECT))
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_encode: unknown flags 0x%x", flags);
  const bool direct = flags & NDGI_HTRAIN_DIRECT, rounded = flags & NDGI_HTRAIN_BCSIM;
  if (direct && (rounded || st->codec != NDGI_CODEC_BC4))
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_encode: DIRECT needs a BC4-layout state and excludes BCSIM");
  if (codec != NDGI_CODEC_BC4 && codec != NDGI_CODEC_BC7)
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_encode: codec %d", codec);
  if (mlp_out && mlp_dtype != NDGI_DTYPE_F32 && mlp_dtype != NDGI_DTYPE_F16)
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_encode: bad dtype");
  const uintptr_t al = codec == NDGI_CODEC_BC7 ? 15u : 7u;
  if (((uintptr_t)fuv_out & al) || ((uintptr_t)fuvt_out & al))
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_encode: block outputs must be aligned to a block");
  const HybTrainDims d = htd_of(st);
  if (model < 0 || model >= d.M) return fail(NDGI_ERR_INVALID_ARG, "hybrid_encode: model %d of %d", model, d.M);
  const float* P = st->params + (int64_t)model * d.o_mlp;
  const float* mlp = st->params + (int64_t)d.M * d.o_mlp + (int64_t)model * (d.n - d.o_mlp);
  TexSrc S = {};
  S.codec = d.codec;
  S.kind = direct ? kSrcDirect : (rounded ? kSrcRounded : kSrcLerp);
  const int per_fp = codec == NDGI_CODEC_BC7 ? 1 : 4;   // blocks per footprint
  if (fuv_out) {
    S.ep = P;
    S.w = P + d.o_uvw;
    S.W = d.W;
    S.H = d.H;
    rc = launch_encode(S, codec, (int64_t)(d.H / 4) * (d.W / 4) * per_fp, fuv_out, c->n_cu, s);
    if (rc) return rc;
  }
  if (fuvt_out) {
    S.ep = P + d.o_tep;
    S.w = P + d.o_tw;
    S.W = d.Gu;
    S.H = d.Gv;
    rc = launch_encode(S, codec, (int64_t)d.S * (d.Gv / 4) * (d.Gu / 4) * per_fp, fuvt_out, c->n_cu, s);
    if (rc) return rc;
  }
  if (fut_out)
    hipLaunchKernelGGL(k_quant8, dim3(grid_of((int64_t)d.Tt * d.U * 2, 1024)), dim3(256), 0, s, P + d.o_ut, fut_out,
                       (int64_t)d.Tt * d.U * 2);
  if (fvt_out)
    hipLaunchKernelGGL(k_quant8, dim3(grid_of((int64_t)d.Tt * d.V * 2, 1024)), dim3(256), 0, s, P + d.o_vt, fvt_out,
                       (int64_t)d.Tt * d.V * 2);
  NDGI_HIP(hipGetLastError());
  if (mlp_out) return launch_convert(c, mlp, mlp_out, mlp_dtype, d.n - d.o_mlp, s);
  return NDGI_OK;
}

int ndgi_hybrid_import(ndgi_ctx* c, const ndgi_hybrid_model* m, ndgi_hybrid_train_state* st, int32_t model,
                       hipStream_t s) {
  clear_error();
  if (!c) return fail(NDGI_ERR_INVALID_ARG, "hybrid_import: ctx is NULL");
  int rc = check_htrain(st, "hybrid_import");
  if (rc) return rc;
  rc = check_hybrid(m, "hybrid_import");
  if (rc) return rc;
  if (st->codec != NDGI_CODEC_BC4)
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_import: the state must have the BC4 layout (a value per texel and "
                                      "channel)");
  if (m->W != st->W || m->H != st->H || m->Gu != st->Gu || m->Gv != st->Gv || m->S != st->S || m->U != st->U ||
      m->V != st->V || m->Tt != st->Tt || m->hidden != st->hidden)
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_import: model and state sizes differ");
  const HybTrainDims d = htd_of(st);
  if (model < 0 || model >= d.M) return fail(NDGI_ERR_INVALID_ARG, "hybrid_import: model %d of %d", model, d.M);
  float* P = st->params + (int64_t)model * d.o_mlp;
  float* mlp = st->params + (int64_t)d.M * d.o_mlp + (int64_t)model * (d.n - d.o_mlp);
  const int64_t ep_uv = d.o_uvw / 2, ep_uvt = (d.o_tw - d.o_tep) / 2;
  hipLaunchKernelGGL(k_fill_ep01, dim3(grid_of(ep_uv, c->n_cu * 16)), dim3(256), 0, s, P, ep_uv);
  hipLaunchKernelGGL(k_fill_ep01, dim3(grid_of(ep_uvt, c->n_cu * 16)), dim3(256), 0, s, P + d.o_tep, ep_uvt);
  rc = launch_import_map(m->fuv, m->codec, d.W, d.H, 1, P + d.o_uvw, c->n_cu, s);
  if (rc) return rc;
  rc = launch_import_map(m->fuvt, m->codec, d.Gu, d.Gv, d.S, P + d.o_tw, c->n_cu, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_unit8, dim3(grid_of((int64_t)d.Tt * d.U * 2, 1024)), dim3(256), 0, s, m->fut, P + d.o_ut,
                     (int64_t)d.Tt * d.U * 2);
  hipLaunchKernelGGL(k_unit8, dim3(grid_of((int64_t)d.Tt * d.V * 2, 1024)), dim3(256), 0, s, m->fvt, P + d.o_vt,
                     (int64_t)d.Tt * d.V * 2);
  hipLaunchKernelGGL(k_to_f32, dim3(grid_of(d.n - d.o_mlp, 64)), dim3(256), 0, s, m->mlp, m->mlp_dtype, mlp,
                     d.n - d.o_mlp);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

int ndgi_hybrid_normalize_target(ndgi_ctx* c, const uint16_t* target, int32_t frames, int32_t W, int32_t H,
                                 float gamma, float* out, double* means, hipStream_t s) {
  clear_error();
  if (!c || !target || !out || !means) return fail(NDGI_ERR_INVALID_ARG, "hybrid_normalize_target: NULL argument");
  if (frames < 1 || frames > 65535 || W < 1 || H < 1 || !(gamma > 0.0f))
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_normalize_target: bad sizes or gamma");
  const int64_t texels = (int64_t)W * H;
  for (int i = 0; i < frames * 3; i += 64)
    hipLaunchKernelGGL(k_zero_d, dim3(1), dim3(64), 0, s, means + i, min(64, frames * 3 - i));
  hipLaunchKernelGGL(k_norm_sum, dim3((unsigned)((texels + kNormChunk - 1) / kNormChunk), frames), dim3(256), 0, s,
                     target, texels, 1.0f / gamma, means);
  hipLaunchKernelGGL(k_norm_apply, dim3(grid_of(texels * 3 * frames, c->n_cu * 16)), dim3(256), 0, s, target, texels,
                     frames, 1.0f / gamma, means, out);
  hipLaunchKernelGGL(k_norm_means, dim3(1), dim3(256), 0, s, means, frames * 3, texels);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

int ndgi_hybrid_restore(ndgi_ctx* c, const void* pred, int32_t pred_dtype, int64_t texels, const double* mean3,
                        float gamma, float* out, hipStream_t s) {
  clear_error();
  if (!c || !pred || !mean3 || !out) return fail(NDGI_ERR_INVALID_ARG, "hybrid_restore: NULL argument");
  if (texels < 0 || !(gamma > 0.0f) || (pred_dtype != NDGI_DTYPE_F32 && pred_dtype != NDGI_DTYPE_F16))
    return fail(NDGI_ERR_INVALID_ARG, "hybrid_restore: bad arguments");
  if (texels == 0) return NDGI_OK;
  hipLaunchKernelGGL(k_restore, dim3(grid_of(texels * 3, c->n_cu * 16)), dim3(256), 0, s, pred, pred_dtype, texels,
                     mean3, gamma, out);
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

}  // extern "C"
