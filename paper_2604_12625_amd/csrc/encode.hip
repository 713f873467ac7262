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
//
// * BC7 with several modes (Sec. 3.4: the BC7 compression may pick among the format's modes): after the
//   mode-6 search, every block tries mode 5 under each of its 4 rotations and mode 4 under
//   each rotation and both index selections, and keeps the candidate of least summed squared
//   error (ties: mode 6, then mode 5 by rotation, then mode 4 by rotation then selection).  A
//   rotation r > 0 encodes the texels with channel r - 1 and channel 3 exchanged.  Modes 5
//   and 4 fit their colour (3 channels) and alpha (1 channel) endpoints apart, each by the
//   same fixed search at its endpoint precision n and index width b: (1) the bounding-box
//   diagonal (one channel: its minimum and maximum), each 8-bit target quantised to the
//   n-bit value whose expansion is nearest (ties to the lower; the candidates are
//   round(x (2^n - 1) / 255) and its neighbours); (2) twice, the least-squares endpoints of
//   the current indices, quantised as in (1); (3) best-improvement local search at steps
//   2^(n - 4) .. 1 over each value of each endpoint -s and +s, then (several channels) all
//   values of one endpoint -s and +s, at most 64 rounds per step; (4) the anchor swap of
//   endpoints and indices J -> 2^b - 1 - J when texel 0's index has its top bit set.
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

// ------------------------------------------------------------ BC7 modes 4 and 5 (subsets)
__device__ __forceinline__ int bc7_xpand(int v, int n) { return n < 8 ? (v << (8 - n)) | (v >> (2 * n - 8)) : v; }

// The n-bit value whose expansion is nearest to the 8-bit target x (ties to the lower).
template <int N>
__device__ __forceinline__ int bc7_quant(int x) {
  constexpr int top = (1 << N) - 1;
  const int g = min(max((x * top + 127) / 255, 0), top);
  int best = 0, bd = INT_MAX;
#pragma unroll
  for (int dv = -1; dv <= 1; ++dv) {
    const int v = min(max(g + dv, 0), top);
    const int d = abs(bc7_xpand(v, N) - x);
    if (d < bd || (d == bd && v < best)) {
      best = v;
      bd = d;
    }
  }
  return best;
}

template <int C>
struct SubRes {
  int v0[C], v1[C], sse, J;
};

// Index fit of endpoints (n-bit values v0, v1) with b-bit indices: J = this lane's texel's
// best index (the lowest on ties; lane (s, g) tries indices PER g .. PER g + PER - 1); returns
// the block's summed squared error in every lane.
template <int C, int N, int IB>
__device__ __forceinline__ int sub_fit(const int X[C], const int v0[C], const int v1[C], int lane, int& J) {
  constexpr int PER = (1 << IB) / 4;
  int E0[C], E1[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    E0[c] = bc7_xpand(v0[c], N);
    E1[c] = bc7_xpand(v1[c], N);
  }
  int best = INT_MAX, bj = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int j = PER * (lane & 3) + k;
    const int w = (64 * j + ((1 << IB) - 1) / 2) / ((1 << IB) - 1);   // the format's weight table
    int d = 0;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int e = (((64 - w) * E0[c] + w * E1[c] + 32) >> 6) - X[c];
      d += e * e;
    }
    if (d < best) {
      best = d;
      bj = j;
    }
  }
#pragma unroll
  for (int off = 1; off < 4; off <<= 1) {
    const int ob = __shfl_xor(best, off, 64), oj = __shfl_xor(bj, off, 64);
    if (ob < best || (ob == best && oj < bj)) {
      best = ob;
      bj = oj;
    }
  }
  J = bj;
  return wave_isum((lane & 3) == 0 ? best : 0);
}

template <int C, int N, int IB>
__device__ __forceinline__ void sub_take(SubRes<C>& cur, const int X[C], const int v0[C], const int v1[C], int lane) {
  int J;
  const int sse = sub_fit<C, N, IB>(X, v0, v1, lane, J);
  if (sse < cur.sse) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      cur.v0[c] = v0[c];
      cur.v1[c] = v1[c];
    }
    cur.sse = sse;
    cur.J = J;
  }
}

template <int C, int N, int IB>
__device__ SubRes<C> sub_search(const int X[C], int lane) {
  constexpr int top = (1 << N) - 1;
  SubRes<C> cur;
  cur.sse = INT_MAX;
  cur.J = 0;
#pragma unroll
  for (int c = 0; c < C; ++c) cur.v0[c] = cur.v1[c] = 0;
  // (1) bounding-box diagonal
  {
    int lo[C], hi[C], A[C], B[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      int mn = X[c], mx = X[c];
#pragma unroll
      for (int off = 4; off < 64; off <<= 1) {
        mn = min(mn, __shfl_xor(mn, off, 64));
        mx = max(mx, __shfl_xor(mx, off, 64));
      }
      lo[c] = mn;
      hi[c] = mx;
    }
    if constexpr (C > 1) {
      int D[C], var[C];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int sum = wave_isum((lane & 3) == 0 ? X[c] : 0);
        D[c] = 16 * X[c] - sum;
        var[c] = wave_isum((lane & 3) == 0 ? D[c] * D[c] : 0);
      }
      int ref = 0;
#pragma unroll
      for (int c = 1; c < C; ++c)
        if (var[c] > var[ref]) ref = c;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const int cov = wave_isum((lane & 3) == 0 ? D[c] * D[ref] : 0);
        A[c] = cov >= 0 ? lo[c] : hi[c];
        B[c] = cov >= 0 ? hi[c] : lo[c];
      }
    } else {
      A[0] = lo[0];
      B[0] = hi[0];
    }
    int q0[C], q1[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      q0[c] = bc7_quant<N>(A[c]);
      q1[c] = bc7_quant<N>(B[c]);
    }
    sub_take<C, N, IB>(cur, X, q0, q1, lane);
  }
  // (2) least-squares endpoints of the current indices, twice
#pragma unroll 1
  for (int it = 0; it < 2; ++it) {
    const int w = (64 * cur.J + ((1 << IB) - 1) / 2) / ((1 << IB) - 1), a = 64 - w;
    const bool mine = (lane & 3) == 0;
    const int64_t Aa = wave_isum(mine ? a * a : 0), Bab = wave_isum(mine ? a * w : 0), Cb = wave_isum(mine ? w * w : 0);
    const int64_t det = Aa * Cb - Bab * Bab;
    int q0[C], q1[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int64_t r0 = 64 * (int64_t)wave_isum(mine ? a * X[c] : 0);
      const int64_t r1 = 64 * (int64_t)wave_isum(mine ? w * X[c] : 0);
      int E0, E1;
      if (det > 0) {
        const int64_t n0 = Cb * r0 - Bab * r1, n1 = Aa * r1 - Bab * r0;
        E0 = (int)min(max(floor_div(2 * n0 + det, 2 * det), (int64_t)0), (int64_t)255);
        E1 = (int)min(max(floor_div(2 * n1 + det, 2 * det), (int64_t)0), (int64_t)255);
      } else {
        E0 = bc7_xpand(cur.v0[c], N);
        E1 = bc7_xpand(cur.v1[c], N);
      }
      q0[c] = bc7_quant<N>(E0);
      q1[c] = bc7_quant<N>(E1);
    }
    sub_take<C, N, IB>(cur, X, q0, q1, lane);
  }
  // (3) local search, coarse to fine
  constexpr int NM = 4 * C + (C > 1 ? 4 : 0);
#pragma unroll 1
  for (int st = 1 << (N - 4); st >= 1; st >>= 1) {
#pragma unroll 1
    for (int round = 0; round < 64; ++round) {
      int bsse = INT_MAX, bmove = -1, bJ = 0;
#pragma unroll 1
      for (int mv = 0; mv < NM; ++mv) {
        int v0[C], v1[C];
#pragma unroll
        for (int c = 0; c < C; ++c) {
          v0[c] = cur.v0[c];
          v1[c] = cur.v1[c];
        }
        bool valid = true;
        const int k = mv < 4 * C ? mv / (2 * C) : (mv - 4 * C) >> 1;
        const int cc = mv < 4 * C ? (mv >> 1) % C : C;   // C: every value of the endpoint
        const int dv = (mv & 1) ? st : -st;
#pragma unroll
        for (int c = 0; c < C; ++c)
          if (cc == C || cc == c) {
            if (k) v1[c] += dv;
            else v0[c] += dv;
            const int t = k ? v1[c] : v0[c];
            valid = valid && t >= 0 && t <= top;
          }
        if (!valid) continue;
        int J;
        const int sse = sub_fit<C, N, IB>(X, v0, v1, lane, J);
        if (sse < bsse) {
          bsse = sse;
          bmove = mv;
          bJ = J;
        }
      }
      if (bmove < 0 || bsse >= cur.sse) break;
      const int k = bmove < 4 * C ? bmove / (2 * C) : (bmove - 4 * C) >> 1;
      const int cc = bmove < 4 * C ? (bmove >> 1) % C : C;
      const int dv = (bmove & 1) ? st : -st;
#pragma unroll
      for (int c = 0; c < C; ++c)
        if (cc == C || cc == c) {
          if (k) cur.v1[c] += dv;
          else cur.v0[c] += dv;
        }
      cur.sse = bsse;
      cur.J = bJ;
    }
  }
  // (4) anchor: texel 0's index without its top bit
  if (__shfl(cur.J, 0, 64) >= (1 << (IB - 1))) {
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int t = cur.v0[c];
      cur.v0[c] = cur.v1[c];
      cur.v1[c] = t;
    }
    cur.J = (1 << IB) - 1 - cur.J;
  }
  return cur;
}

// OR value v (< 256) into the 128-bit block (lo, hi) at bit pos.
__device__ __forceinline__ void bc7_put(uint64_t& lo, uint64_t& hi, uint32_t v, int pos) {
  if (pos >= 64) {
    hi |= (uint64_t)v << (pos - 64);
  } else {
    lo |= (uint64_t)v << pos;
    if (pos > 56) hi |= (uint64_t)v >> (64 - pos);
  }
}

// This lane's texel index J into an index set of b-bit indices starting at bit pos (lanes
// of texel s: s = lane >> 2; only the first lane of a texel contributes).
__device__ __forceinline__ void bc7_put_index(uint64_t& lo, uint64_t& hi, int J, int pos, int b, int lane) {
  const int s = lane >> 2;
  if ((lane & 3) == 0) bc7_put(lo, hi, (uint32_t)J, s ? pos + b - 1 + b * (s - 1) : pos);
}

// The winning candidate of modes 4 and 5 for a block.
struct M45 {
  int mode, rot, sel, sse;
  SubRes<3> col;
  SubRes<1> alp;
};

template <int MODE, int SEL>
__device__ __forceinline__ void m45_try(M45& best, const int X[4], int rot, int lane) {
  int Y[4] = {X[0], X[1], X[2], X[3]};
  if (rot) {
    Y[rot - 1] = X[3];
    Y[3] = X[rot - 1];
  }
  SubRes<3> col;
  SubRes<1> alp;
  if constexpr (MODE == 5) {
    col = sub_search<3, 7, 2>(Y, lane);
    alp = sub_search<1, 8, 2>(Y + 3, lane);
  } else if constexpr (SEL == 0) {
    col = sub_search<3, 5, 2>(Y, lane);
    alp = sub_search<1, 6, 3>(Y + 3, lane);
  } else {
    col = sub_search<3, 5, 3>(Y, lane);
    alp = sub_search<1, 6, 2>(Y + 3, lane);
  }
  const int sse = col.sse + alp.sse;
  if (sse < best.sse) {
    best.mode = MODE;
    best.rot = rot;
    best.sel = SEL;
    best.sse = sse;
    best.col = col;
    best.alp = alp;
  }
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
    // modes 5 and 4, each rotation (and, mode 4, index selection): a candidate replaces the
    // block only when strictly better
    M45 alt;
    alt.mode = 6;
    alt.sse = cur.sse;
#pragma unroll 1
    for (int r = 0; r < 4; ++r) m45_try<5, 0>(alt, X, r, lane);
#pragma unroll 1
    for (int r = 0; r < 4; ++r) {
      m45_try<4, 0>(alt, X, r, lane);
      m45_try<4, 1>(alt, X, r, lane);
    }
    if (alt.mode != 6) {   // wave-uniform
      uint64_t lo = 0, hi = 0;
      if (alt.mode == 5) {
        bc7_put_index(lo, hi, alt.col.J, 66, 2, lane);
        bc7_put_index(lo, hi, alt.alp.J, 97, 2, lane);
      } else {
        bc7_put_index(lo, hi, alt.sel ? alt.alp.J : alt.col.J, 50, 2, lane);
        bc7_put_index(lo, hi, alt.sel ? alt.col.J : alt.alp.J, 81, 3, lane);
      }
#pragma unroll
      for (int off = 4; off < 64; off <<= 1) {
        lo |= __shfl_xor(lo, off, 64);
        hi |= __shfl_xor(hi, off, 64);
      }
      if (lane == 0) {
        if (alt.mode == 5) {
          lo |= (uint64_t)((1 << 5) | (alt.rot << 6));
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            bc7_put(lo, hi, (uint32_t)alt.col.v0[c], 8 + 14 * c);
            bc7_put(lo, hi, (uint32_t)alt.col.v1[c], 15 + 14 * c);
          }
          bc7_put(lo, hi, (uint32_t)alt.alp.v0[0], 50);
          bc7_put(lo, hi, (uint32_t)alt.alp.v1[0], 58);
        } else {
          lo |= (uint64_t)((1 << 4) | (alt.rot << 5) | (alt.sel << 7));
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            bc7_put(lo, hi, (uint32_t)alt.col.v0[c], 8 + 10 * c);
            bc7_put(lo, hi, (uint32_t)alt.col.v1[c], 13 + 10 * c);
          }
          bc7_put(lo, hi, (uint32_t)alt.alp.v0[0], 38);
          bc7_put(lo, hi, (uint32_t)alt.alp.v1[0], 44);
        }
        *(u4v*)(out + f * 16) = (u4v){(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32)};
      }
      continue;
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
