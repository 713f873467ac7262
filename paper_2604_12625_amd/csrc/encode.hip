// Block encoders from 8-bit texel values, for the paper's export path (Sec. 3.4, last
// paragraph of Feature Map Compression): after training, F_uv and F_uvt are reconstructed
// from their parameters, quantised to 8 bits and block-compressed; the supplementary
// ablation's "w/o BC simulation" arm compresses a directly optimised map the same way.  The
// paper names no encoder.  Two are built, both integer-only and deterministic:
//
// * BC4 (one channel of 16 texels): the optimum in summed squared error over all 65536
//   endpoint pairs (both palette modes), each texel at its nearest palette entry; ties go to
//   the lowest pair e0 * 256 + e1, and per texel to the lowest selector.  One workgroup per
//   block: thread e0 walks e1 = 0..255 (increasing pair order), skipping the rest of a pair
//   once its partial error exceeds the thread's best; the (error, pair) minimum is then
//   taken over the workgroup.
//
// * BC7 mode 6 (4 channels of 16 texels): its 2^58 endpoint settings are too many to try, so
//   the encoder is a fixed search.  (1) Endpoints at the corners of the texels' bounding box
//   along its principal diagonal: the channel of largest spread is the reference, and a
//   channel runs from its minimum to its maximum when its covariance with the reference is
//   >= 0, else from maximum to minimum.  (2) Both target endpoints quantised for each of the
//   four p-bit pairs, v = clamp(floor((x - p + 1) / 2), 0, 127); a candidate replaces the
//   current block only when strictly better.  (3) Twice: the least-squares endpoints of the
//   current indices (per channel the 2 x 2 normal equations of
//   sum ((64 - w) E0 + w E1 - 64 x)^2, solved exactly in integers, rounded half up, clamped to
//   0..255), quantised as in (2).  (4) Best-improvement local search at steps 8, 4, 2, 1, at
//   most 64 rounds per step, over 22 moves in a fixed order (each 7-bit value of endpoint 0,
//   then of endpoint 1, by -s and +s; all four values of endpoint 0, then of endpoint 1, by
//   -s and +s; the p-bit of endpoint 0, then of endpoint 1, flipped; a move leaving 0..127 is
//   not taken); the first strictly best move is taken while it improves.  (5) When texel 0's
//   index has its top bit set (the anchor index has 3 bits) the endpoints swap and every
//   index J becomes 15 - J, which decodes identically.  Every candidate's indices are
//   refitted: each texel takes its least-error index, the lowest on ties.  One wave per
//   block: lane (s, g) = (lane >> 2, lane & 3) holds texel s and tries indices 4g .. 4g + 3.
#include <climits>

#include "bcsim.hpp"
#include "internal.hpp"

namespace ndgi {

// The 4 channels (0..255) of texel s of footprint f.
__device__ __forceinline__ void src_texel4(const TexSrc& S, int64_t f, int s, int q[4]) {
  if (S.u8) {
#pragma unroll
    for (int c = 0; c < 4; ++c) q[c] = c < S.C ? (int)S.u8[(f * 16 + s) * S.C + c] : 0;
    return;
  }
  const int wb = S.W >> 2;
  const int64_t per = (int64_t)(S.H >> 2) * wb;
  const int64_t sl = f / per, rem = f - sl * per;
  const int x = 4 * (int)(rem % wb) + (s & 3), y = 4 * (int)(rem / wb) + (s >> 2);
  const int cw = S.codec ? 1 : 4;
  map_texel_u8(S.ep + f * 8, S.w + ((sl * S.H + y) * S.W + x) * cw, S.kind, S.codec, q);
}

// --------------------------------------------------------------------------------- BC4
__device__ __forceinline__ void bc4_palette8(int e0, int e1, int p[8]) {
  p[0] = e0;
  p[1] = e1;
  if (e0 > e1) {
#pragma unroll
    for (int j = 1; j <= 6; ++j) p[j + 1] = ((7 - j) * e0 + j * e1 + 3) / 7;
  } else {
#pragma unroll
    for (int j = 1; j <= 4; ++j) p[j + 1] = ((5 - j) * e0 + j * e1 + 2) / 5;
    p[6] = 0;
    p[7] = 255;
  }
}

// Block b: channel b % 4 of footprint b / 4 of a map source, or 16 texels at u8 + 16 b.
__global__ __launch_bounds__(256) void k_encode_bc4(TexSrc S, int64_t n, uint8_t* __restrict__ out) {
  __shared__ int tex[16];
  __shared__ int64_t red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int64_t b = blockIdx.x; b < n; b += gridDim.x) {
    __syncthreads();   // the previous block's readers of tex and red are done
    if (tid < 16) {
      int q[4];
      if (S.u8) {
        q[0] = S.u8[b * 16 + tid];
      } else {
        src_texel4(S, b >> 2, tid, q);
        q[0] = q[b & 3];
      }
      tex[tid] = q[0];
    }
    __syncthreads();
    int X[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) X[s] = tex[s];
    const int e0 = tid;
    int best = INT_MAX, bp = 0;
    for (int e1 = 0; e1 < 256; ++e1) {
      int p[8];
      bc4_palette8(e0, e1, p);
      int sse = 0;
#pragma unroll
      for (int s4 = 0; s4 < 16; s4 += 4) {
        if (sse <= best) {   // else the pair cannot become strictly better
#pragma unroll
          for (int s = s4; s < s4 + 4; ++s) {
            int m = INT_MAX;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const int d = p[k] - X[s];
              m = min(m, d * d);
            }
            sse += m;
          }
        }
      }
      if (sse < best) {
        best = sse;
        bp = e0 * 256 + e1;
      }
    }
    // (error, pair) minimum over the workgroup: the key orders by error, then by pair
    int64_t key = ((int64_t)best << 16) | bp;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const int64_t o = __shfl_xor(key, off, 64);
      key = o < key ? o : key;
    }
    if (lane == 0) red[wave] = key;
    __syncthreads();
    if (tid < 16) {
      int64_t k = red[0];
#pragma unroll
      for (int w = 1; w < 4; ++w) k = red[w] < k ? red[w] : k;
      const int pair = (int)(k & 0xffff), E0 = pair >> 8, E1 = pair & 255;
      int p[8];
      bc4_palette8(E0, E1, p);
      int code = 0, m = INT_MAX;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int d = p[c] - X[tid];
        if (d * d < m) {
          m = d * d;
          code = c;
        }
      }
      // gather the 16 selectors in lanes 0..15 and pack
      uint64_t field = (uint64_t)code << (3 * tid);
#pragma unroll
      for (int off = 8; off > 0; off >>= 1) field |= __shfl_xor(field, off, 16);
      if (tid == 0) {
        const uint32_t lo = (uint32_t)E0 | ((uint32_t)E1 << 8) | ((uint32_t)(field & 0xffffu) << 16);
        const uint32_t hi = (uint32_t)(field >> 16);
        *(uint2*)(out + b * 8) = make_uint2(lo, hi);
      }
    }
  }
}

// ---------------------------------------------------------------------------- BC7 mode 6
// Sum over all 64 lanes, returned in every lane.  Callers pass one texel's value in its
// first lane (lane & 3 == 0) and 0 in the other three.
__device__ __forceinline__ int wave_isum(int v) {
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Index fit of endpoints E0, E1 for the wave's block: J = this lane's texel's best index
// (the lowest on ties); returns the block's summed squared error (the same in every lane).
__device__ __forceinline__ int m6_fit(const int X[4], const int E0[4], const int E1[4], int lane, int& J) {
  int best = INT_MAX, bj = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int j = 4 * (lane & 3) + k;
    const int w = (64 * j + 7) / 15;   // the format's 4-bit weight table
    int d = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int e = (((64 - w) * E0[c] + w * E1[c] + 32) >> 6) - X[c];
      d += e * e;
    }
    if (d < best) {
      best = d;
      bj = j;
    }
  }
#pragma unroll
  for (int off = 1; off < 4; off <<= 1) {   // the texel's 4 lanes: least error, lowest index
    const int ob = __shfl_xor(best, off, 64), oj = __shfl_xor(bj, off, 64);
    if (ob < best || (ob == best && oj < bj)) {
      best = ob;
      bj = oj;
    }
  }
  J = bj;
  return wave_isum((lane & 3) == 0 ? best : 0);
}

struct M6 {
  int v0[4], v1[4], p0, p1, sse, J;
};


// Try (v0, p0, v1, p1): taken when strictly better than the current block.
__device__ __forceinline__ void m6_take(M6& cur, const int X[4], const int v0[4], int p0, const int v1[4], int p1,
                                        int lane) {
  int E0[4], E1[4], J;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    E0[c] = 2 * v0[c] + p0;
    E1[c] = 2 * v1[c] + p1;
  }
  const int sse = m6_fit(X, E0, E1, lane, J);
  if (sse < cur.sse) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      cur.v0[c] = v0[c];
      cur.v1[c] = v1[c];
    }
    cur.p0 = p0;
    cur.p1 = p1;
    cur.sse = sse;
    cur.J = J;
  }
}

// Targets A, B (8-bit, per channel) quantised for the four p-bit pairs.
__device__ __forceinline__ void m6_quantised(M6& cur, const int X[4], const int A[4], const int B[4], int lane) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int p0 = q >> 1, p1 = q & 1;
    int v0[4], v1[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      v0[c] = min(max((A[c] - p0 + 1) >> 1, 0), 127);
      v1[c] = min(max((B[c] - p1 + 1) >> 1, 0), 127);
    }
    m6_take(cur, X, v0, p0, v1, p1, lane);
  }
}

__device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {   // b > 0
  const int64_t q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}

__global__ __launch_bounds__(256) void k_encode_bc7(TexSrc S, int64_t n, uint8_t* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int s = lane >> 2;
  const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t f = wave0; f < n; f += stride) {
    int X[4];
    src_texel4(S, f, s, X);
    M6 cur;
    cur.sse = INT_MAX;
    cur.J = 0;
    cur.p0 = cur.p1 = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) cur.v0[c] = cur.v1[c] = 0;
    // (1)-(2): the bounding box's principal diagonal
    {
      int sum[4], lo[4], hi[4], D[4], var[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        int a = (lane & 3) == 0 ? X[c] : 0;
        sum[c] = wave_isum(a);
        int mn = X[c], mx = X[c];
#pragma unroll
        for (int off = 4; off < 64; off <<= 1) {
          mn = min(mn, __shfl_xor(mn, off, 64));
          mx = max(mx, __shfl_xor(mx, off, 64));
        }
        lo[c] = mn;
        hi[c] = mx;
        D[c] = 16 * X[c] - sum[c];
        var[c] = wave_isum((lane & 3) == 0 ? D[c] * D[c] : 0);
      }
      int ref = 0;
#pragma unroll
      for (int c = 1; c < 4; ++c)
        if (var[c] > var[ref]) ref = c;
      int A[4], B[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int cov = wave_isum((lane & 3) == 0 ? D[c] * D[ref] : 0);
        A[c] = cov >= 0 ? lo[c] : hi[c];
        B[c] = cov >= 0 ? hi[c] : lo[c];
      }
      m6_quantised(cur, X, A, B, lane);
    }
    // (3): least-squares endpoints of the current indices, twice
#pragma unroll 1
    for (int it = 0; it < 2; ++it) {
      const int w = (64 * cur.J + 7) / 15, a = 64 - w;
      const bool mine = (lane & 3) == 0;
      const int64_t Aa = wave_isum(mine ? a * a : 0), Bab = wave_isum(mine ? a * w : 0), Cb = wave_isum(mine ? w * w : 0);
      const int64_t det = Aa * Cb - Bab * Bab;
      int E0[4], E1[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t r0 = 64 * (int64_t)wave_isum(mine ? a * X[c] : 0);
        const int64_t r1 = 64 * (int64_t)wave_isum(mine ? w * X[c] : 0);
        if (det > 0) {
          const int64_t n0 = Cb * r0 - Bab * r1, n1 = Aa * r1 - Bab * r0;
          E0[c] = (int)min(max(floor_div(2 * n0 + det, 2 * det), (int64_t)0), (int64_t)255);
          E1[c] = (int)min(max(floor_div(2 * n1 + det, 2 * det), (int64_t)0), (int64_t)255);
        } else {
          E0[c] = 2 * cur.v0[c] + cur.p0;
          E1[c] = 2 * cur.v1[c] + cur.p1;
        }
      }
      m6_quantised(cur, X, E0, E1, lane);
    }
    // (4): local search, coarse to fine
#pragma unroll 1
    for (int st = 8; st >= 1; st >>= 1) {
#pragma unroll 1
      for (int round = 0; round < 64; ++round) {
        int bsse = INT_MAX, bmove = -1, bJ = 0;
#pragma unroll 1
        for (int mv = 0; mv < 22; ++mv) {
          int v0[4], v1[4], p0 = cur.p0, p1 = cur.p1;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            v0[c] = cur.v0[c];
            v1[c] = cur.v1[c];
          }
          bool valid = true;
          if (mv < 16) {            // one value: endpoint mv >> 3, channel (mv >> 1) & 3, sign mv & 1
            const int k = mv >> 3, c = (mv >> 1) & 3, dv = (mv & 1) ? st : -st;
            int* v = k ? v1 : v0;
#pragma unroll
            for (int cc = 0; cc < 4; ++cc)
              if (cc == c) {
                v[cc] += dv;
                valid = v[cc] >= 0 && v[cc] <= 127;
              }
          } else if (mv < 20) {     // all four values of endpoint (mv - 16) >> 1
            const int k = (mv - 16) >> 1, dv = (mv & 1) ? st : -st;
            int* v = k ? v1 : v0;
#pragma unroll
            for (int cc = 0; cc < 4; ++cc) {
              v[cc] += dv;
              valid = valid && v[cc] >= 0 && v[cc] <= 127;
            }
          } else if (mv == 20) {
            p0 ^= 1;
          } else {
            p1 ^= 1;
          }
          if (!valid) continue;
          int E0[4], E1[4], J;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            E0[c] = 2 * v0[c] + p0;
            E1[c] = 2 * v1[c] + p1;
          }
          const int sse = m6_fit(X, E0, E1, lane, J);
          if (sse < bsse) {
            bsse = sse;
            bmove = mv;
            bJ = J;
          }
        }
        if (bmove < 0 || bsse >= cur.sse) break;
        if (bmove < 16) {
          const int k = bmove >> 3, c = (bmove >> 1) & 3, dv = (bmove & 1) ? st : -st;
#pragma unroll
          for (int cc = 0; cc < 4; ++cc)
            if (cc == c) {
              if (k) cur.v1[cc] += dv;
              else cur.v0[cc] += dv;
            }
        } else if (bmove < 20) {
          const int k = (bmove - 16) >> 1, dv = (bmove & 1) ? st : -st;
#pragma unroll
          for (int cc = 0; cc < 4; ++cc) {
            if (k) cur.v1[cc] += dv;
            else cur.v0[cc] += dv;
          }
        } else if (bmove == 20) {
          cur.p0 ^= 1;
        } else {
          cur.p1 ^= 1;
        }
        cur.sse = bsse;
        cur.J = bJ;
      }
    }
    // (5): anchor and packing; texel s's index sits in lane 4 s
    const int j0 = __shfl(cur.J, 0, 64);
    const bool swap = j0 >= 8;
    const int J = swap ? 15 - cur.J : cur.J;
    uint64_t hi = s ? (uint64_t)J << (4 * s) : (uint64_t)J << 1;
    hi = (lane & 3) == 0 ? hi : 0;
#pragma unroll
    for (int off = 4; off < 64; off <<= 1) hi |= __shfl_xor(hi, off, 64);
    if (lane == 0) {
      const int* a = swap ? cur.v1 : cur.v0;
      const int* z = swap ? cur.v0 : cur.v1;
      const int pa = swap ? cur.p1 : cur.p0, pz = swap ? cur.p0 : cur.p1;
      uint64_t lo = 0x40;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        lo |= (uint64_t)a[c] << (7 + 14 * c);
        lo |= (uint64_t)z[c] << (14 + 14 * c);
      }
      lo |= (uint64_t)pa << 63;
      hi |= (uint64_t)pz;
      *(u4v*)(out + f * 16) = (u4v){(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32)};
    }
  }
}

int launch_encode(const TexSrc& S, int codec, int64_t n, uint8_t* out, int n_cu, hipStream_t s) {
  if (n <= 0) return NDGI_OK;
  if (codec == NDGI_CODEC_BC7) {
    const int64_t wgs = (n + 3) / 4, cap = (int64_t)n_cu * 16;
    hipLaunchKernelGGL(k_encode_bc7, dim3((unsigned)(wgs < cap ? wgs : cap)), dim3(256), 0, s, S, n, out);
  } else {
    const int64_t cap = (int64_t)n_cu * 8;
    hipLaunchKernelGGL(k_encode_bc4, dim3((unsigned)(n < cap ? n : cap)), dim3(256), 0, s, S, n, out);
  }
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

}  // namespace ndgi

using namespace ndgi;

extern "C" {

int ndgi_bc4_encode_blocks(const uint8_t* texels, int64_t n, uint8_t* out, hipStream_t s) {
  clear_error();
  if (n < 0) return fail(NDGI_ERR_INVALID_ARG, "bc4_encode_blocks: n < 0");
  if (n > 0 && (!texels || !out)) return fail(NDGI_ERR_INVALID_ARG, "bc4_encode_blocks: NULL pointer");
  if (((uintptr_t)out & 7u) != 0) return fail(NDGI_ERR_INVALID_ARG, "bc4_encode_blocks: out not 8-byte aligned");
  int dev = 0, n_cu = 0;
  NDGI_HIP(hipGetDevice(&dev));
  NDGI_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  TexSrc S = {};
  S.u8 = texels;
  S.C = 1;
  return launch_encode(S, NDGI_CODEC_BC4, n, out, n_cu, s);
}

int ndgi_bc7_encode_blocks(const uint8_t* texels, int64_t n, uint8_t* out, hipStream_t s) {
  clear_error();
  if (n < 0) return fail(NDGI_ERR_INVALID_ARG, "bc7_encode_blocks: n < 0");
  if (n > 0 && (!texels || !out)) return fail(NDGI_ERR_INVALID_ARG, "bc7_encode_blocks: NULL pointer");
  if (((uintptr_t)out & 15u) != 0) return fail(NDGI_ERR_INVALID_ARG, "bc7_encode_blocks: out not 16-byte aligned");
  int dev = 0, n_cu = 0;
  NDGI_HIP(hipGetDevice(&dev));
  NDGI_HIP(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  TexSrc S = {};
  S.u8 = texels;
  S.C = 4;
  return launch_encode(S, NDGI_CODEC_BC7, n, out, n_cu, s);
}

}  // extern "C"
