// Spatially binned random-access decode.
//
// Random (u, v, t) queries taken in arrival order each touch their own 128-byte lines for
// the four BC4 footprints and the eight grid nodes they read, so a direct decode moves
// many times the bytes it uses.  Here the queries are first counting-sorted by the tile
// of TS x TS texels that holds the upper-left texel of their bilinear footprint.  The
// sorted queries of each tile are split into work items of at most kPiece queries; for
// each item the workgroup decodes the tile's BC4 footprints (plus a one-footprint halo on
// the right and bottom) into LDS once and orders the item's queries by time key, so each
// query reads its four texels from LDS and its grid nodes from a one- or two-key window
// that stays in cache, and writes its RGB at its original index.  The per-query
// arithmetic is the direct decode's, so both give the same bits.
#include <algorithm>

#include "device.hpp"
#include "internal.hpp"

namespace ndgi {

constexpr int kSortWgs = 512;       // workgroups of the counting sort (1024 threads each)
static_assert(kSortWgs % 8 == 0, "sort slices are spread evenly over the 8 XCDs");
constexpr int kBatch = 16;          // queries per thread whose loads are in flight together
constexpr int kSortThreads = 1024;
constexpr int kMaxBins = 16384;     // LDS histogram capacity (64 KiB)
constexpr int kPiece = 2048;        // at most this many queries per decode work item
constexpr int kMaxKeys = 1024;      // largest T the host accepts
constexpr int kStartBins = 1024;    // bins per workgroup of the bin-start scan
constexpr int kStartWgs = kMaxBins / kStartBins;

struct BinGeom {
  int ts_log2;      // tile side = 1 << ts_log2 texels (5 or 6)
  int ntx, nty;     // tiles per row / column
  int galign;       // 1: tiles of 8 x 8 grid cells (grid at a quarter of the texel resolution)
};

static bool bin_geom(const ndgi_model& m, BinGeom& g) {
  for (g.ts_log2 = 5; g.ts_log2 <= 6; ++g.ts_log2) {
    g.galign = g.ts_log2 == 5 && m.W == 4 * m.Gw && m.H == 4 * m.Gh;
    g.ntx = g.galign ? (m.Gw + 7) >> 3 : (m.W + (1 << g.ts_log2) - 1) >> g.ts_log2;
    g.nty = g.galign ? (m.Gh + 7) >> 3 : (m.H + (1 << g.ts_log2) - 1) >> g.ts_log2;
    if ((int64_t)g.ntx * g.nty <= kMaxBins) return true;
  }
  return false;
}

// Tile of a query.  Texel tiles: the tile holding the clamped upper-left texel of its
// bilinear footprint (coordinates outside the map, and NaN, clamp to an edge texel as the
// decode does), so the footprint lies inside the tile plus one texel to the right and
// below.  Grid-aligned tiles (grid at a quarter of the texel resolution): the tile of 8 x 8
// cells holding the upper-left grid node of the query, so the query reads nodes 8k..8k+8
// of each axis (9, where a texel tile's 32 texels reach 10) and texels 32k+1..32k+34 (the
// region of the texel tile 32k..32k+31 plus its halo).
__device__ __forceinline__ int query_bin(float u, float v, const ndgi_model& m, const BinGeom& bg) {
  if (bg.galign) return (coord_axis(v, m.Gh).i0 >> 3) * bg.ntx + (coord_axis(u, m.Gw).i0 >> 3);
  const Axis ax = coord_axis(u, m.W), ay = coord_axis(v, m.H);
  return (ay.i0 >> bg.ts_log2) * bg.ntx + (ax.i0 >> bg.ts_log2);
}

// Slice of the queries handled by a sort workgroup.  Workgroups are dispatched to the 8
// XCDs round-robin; slices are numbered so that each XCD takes kSortWgs / 8 consecutive
// slices.  A bin's records are stored slice after slice, so neighbouring slices' short
// runs share cache lines, which then fill up in one L2 instead of being written back
// half-full from two.
__device__ __forceinline__ int sort_slice() {
  return (int)(blockIdx.x & 7) * (kSortWgs / 8) + (int)(blockIdx.x >> 3);
}

// counts[s][bin] = queries of slice s (a contiguous run of `slice` queries)
// that fall in bin.
__global__ __launch_bounds__(kSortThreads) void k_bin_count(ndgi_model m, BinGeom bg, const float* __restrict__ uvt,
                                                            int64_t n, int64_t slice, int32_t* __restrict__ counts) {
  __shared__ int32_t hist[kMaxBins];
  const int nbins = bg.ntx * bg.nty;
  for (int i = threadIdx.x; i < nbins; i += kSortThreads) hist[i] = 0;
  __syncthreads();
  const int sl = sort_slice();
  const int64_t lo = (int64_t)sl * slice, hi = min(n, lo + slice);
  // loads of kBatch queries are issued before any is used, so they are in flight together
  for (int64_t base = lo + threadIdx.x; base < hi; base += kSortThreads * kBatch) {
    float u[kBatch], v[kBatch];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int64_t q = min(base + (int64_t)kSortThreads * k, hi - 1);
      u[k] = uvt[q * 3];
      v[k] = uvt[q * 3 + 1];
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k)
      if (base + (int64_t)kSortThreads * k < hi) atomicAdd(&hist[query_bin(u[k], v[k], m, bg)], 1);
  }
  __syncthreads();
  int32_t* row = counts + (int64_t)sl * nbins;
  for (int i = threadIdx.x; i < nbins; i += kSortThreads) row[i] = hist[i];
}

// Per bin: exclusive prefix of counts over the sort workgroups, in place, and the bin's
// total into start[bin].  A workgroup takes 32 bins; eight groups of its threads each take
// an eighth of the sort rows, with all of a thread's loads issued together, and the eighth
// sums are combined through LDS.  The workgroup's bin totals and work items (ceil(total /
// kPiece) per bin) are summed into wsums[2 g], wsums[2 g + 1] for workgroup g.
constexpr int kColParts = 8, kColBins = 256 / kColParts, kColRows = kSortWgs / kColParts;
__global__ __launch_bounds__(256) void k_bin_colscan(int32_t* __restrict__ counts, int nbins,
                                                     int32_t* __restrict__ start, int32_t* __restrict__ wsums) {
  __shared__ int32_t part[kColParts][kColBins];
  const int bl = threadIdx.x & (kColBins - 1), pr = threadIdx.x / kColBins;
  const int b = blockIdx.x * kColBins + bl;
  const bool live = b < nbins;
  const int bc = live ? b : nbins - 1;
  int32_t c[kColRows];
#pragma unroll
  for (int r = 0; r < kColRows; ++r) c[r] = counts[(int64_t)(pr * kColRows + r) * nbins + bc];
  int32_t s = 0;
#pragma unroll
  for (int r = 0; r < kColRows; ++r) s += c[r];
  part[pr][bl] = s;
  __syncthreads();
  int32_t run = 0;
  for (int q = 0; q < pr; ++q) run += part[q][bl];
  if (live) {
#pragma unroll
    for (int r = 0; r < kColRows; ++r) {
      counts[(int64_t)(pr * kColRows + r) * nbins + b] = run;
      run += c[r];
    }
  }
  if (pr == kColParts - 1) {   // the last 32 threads, lanes 32..63 of the last wave
    if (live) start[b] = run;
    int32_t t = live ? run : 0, ti = live ? (run + kPiece - 1) / kPiece : 0;
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) {
      t += __shfl_xor(t, off, 32);
      ti += __shfl_xor(ti, off, 32);
    }
    if (bl == 0) {
      wsums[2 * blockIdx.x] = t;
      wsums[2 * blockIdx.x + 1] = ti;
    }
  }
}

// start[0..nbins) := exclusive prefix of the bin totals, start[nbins] := n;
// items[b] := exclusive prefix of the work items per bin (ceil(count / kPiece)),
// items[nbins] := total; item_bin[i] := the bin of work item i.  Workgroup w takes bins
// [w kStartBins, (w + 1) kStartBins), one per thread: its offsets start from the sums of
// the column-scan workgroups before its block (wsums, one pair per 32 bins, reduced with
// wave shuffles and LDS), and its own bins are scanned with wave shuffles and the 16 wave
// sums.  Each thread reads and rewrites only its own bin's entry.
__global__ __launch_bounds__(kStartBins) void k_bin_starts(int32_t* __restrict__ start, int32_t* __restrict__ items,
                                                           int32_t* __restrict__ item_bin, int nbins, int32_t n,
                                                           const int32_t* __restrict__ wsums) {
  static_assert(kStartBins % kColBins == 0 && kStartBins / kColBins * kStartWgs <= kStartBins,
                "the column-scan sums before any block fit one per thread");
  __shared__ int32_t wsum[16], wsumi[16], bsum[2];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int b = blockIdx.x * kStartBins + threadIdx.x;
  // bins and items of the blocks before this one: thread t < (column-scan workgroups before
  // the block) takes workgroup t's pair
  {
    const int before = (int)blockIdx.x * (kStartBins / kColBins);
    int32_t p = (int)threadIdx.x < before ? wsums[2 * threadIdx.x] : 0;
    int32_t pi = (int)threadIdx.x < before ? wsums[2 * threadIdx.x + 1] : 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      p += __shfl_xor(p, off, 64);
      pi += __shfl_xor(pi, off, 64);
    }
    if (threadIdx.x < 2) bsum[threadIdx.x] = 0;
    __syncthreads();
    if (lane == 0 && p) atomicAdd(&bsum[0], p);
    if (lane == 0 && pi) atomicAdd(&bsum[1], pi);
    __syncthreads();
  }
  const int32_t base = bsum[0], basei = bsum[1];
  const int32_t c = b < nbins ? start[b] : 0;
  const int32_t ci = (c + kPiece - 1) / kPiece;
  int32_t incl = c, incli = ci;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t o = __shfl_up(incl, off, 64), oi = __shfl_up(incli, off, 64);
    if (lane >= off) {
      incl += o;
      incli += oi;
    }
  }
  if (lane == 63) {
    wsum[wave] = incl;
    wsumi[wave] = incli;
  }
  __syncthreads();
  int32_t run = base + incl - c, runi = basei + incli - ci;
  for (int q = 0; q < wave; ++q) {
    run += wsum[q];
    runi += wsumi[q];
  }
  if (b < nbins) {
    start[b] = run;
    items[b] = runi;
    for (int j = 0; j < ci; ++j) item_bin[runi + j] = b;
  }
  if (b == nbins - 1) {   // the map's last bin closes both tables
    start[nbins] = n;
    items[nbins] = runi + ci;
  }
}

// Scatter: every query of sort workgroup wg goes to the next free slot of its bin; a
// slot holds (u, v, t, original index).  The order inside a bin is unspecified; each
// query's result does not depend on it.
__global__ __launch_bounds__(kSortThreads) void k_bin_scatter(ndgi_model m, BinGeom bg, const float* __restrict__ uvt,
                                                              int64_t n, int64_t slice,
                                                              const int32_t* __restrict__ counts,
                                                              const int32_t* __restrict__ start,
                                                              float4* __restrict__ sorted) {
  __shared__ int32_t pos[kMaxBins];
  const int nbins = bg.ntx * bg.nty;
  const int sl = sort_slice();
  const int32_t* row = counts + (int64_t)sl * nbins;
  for (int i = threadIdx.x; i < nbins; i += kSortThreads) pos[i] = start[i] + row[i];
  __syncthreads();
  const int64_t lo = (int64_t)sl * slice, hi = min(n, lo + slice);
  for (int64_t base = lo + threadIdx.x; base < hi; base += kSortThreads * kBatch) {
    float u[kBatch], v[kBatch], t[kBatch];
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int64_t q = min(base + (int64_t)kSortThreads * k, hi - 1);
      u[k] = uvt[q * 3];
      v[k] = uvt[q * 3 + 1];
      t[k] = uvt[q * 3 + 2];
    }
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int64_t q = base + (int64_t)kSortThreads * k;
      if (q < hi) {
        const int p = atomicAdd(&pos[query_bin(u[k], v[k], m, bg)], 1);
        sorted[p] = make_float4(u[k], v[k], t[k], __builtin_bit_cast(float, (uint32_t)q));
      }
    }
  }
}

// Bytes i of a, b, c, d packed into one word, for each i: a 4 x 4 byte transpose.
__device__ __forceinline__ void transpose4(uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t o[4]) {
  const uint32_t ab_lo = __builtin_amdgcn_perm(b, a, 0x05010400u);   // a0 b0 a1 b1
  const uint32_t ab_hi = __builtin_amdgcn_perm(b, a, 0x07030602u);   // a2 b2 a3 b3
  const uint32_t cd_lo = __builtin_amdgcn_perm(d, c, 0x05010400u);
  const uint32_t cd_hi = __builtin_amdgcn_perm(d, c, 0x07030602u);
  o[0] = __builtin_amdgcn_perm(cd_lo, ab_lo, 0x05040100u);           // a0 b0 c0 d0
  o[1] = __builtin_amdgcn_perm(cd_lo, ab_lo, 0x07060302u);
  o[2] = __builtin_amdgcn_perm(cd_hi, ab_hi, 0x05040100u);
  o[3] = __builtin_amdgcn_perm(cd_hi, ab_hi, 0x07060302u);
}

// Exclusive prefix sum of a[0..len) in place by one wave (len <= 64 * 16).
__device__ __forceinline__ void wave_exclusive_scan(int32_t* a, int len, int lane) {
  const int per = (len + 63) >> 6;
  const int lo = lane * per, hi = min(len, lo + per);
  int32_t s = 0;
  for (int i = lo; i < hi; ++i) s += a[i];
  int32_t incl = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  int32_t run = incl - s;
  for (int i = lo; i < hi; ++i) {
    const int32_t c = a[i];
    a[i] = run;
    run += c;
  }
}

// Decode of the sorted queries.  Per work item the workgroup
//  * decodes the tile region into LDS: R = TS + 4 texels a side (the tile plus one
//    footprint of halo), 8 bytes per texel (channel c in byte c);
//  * orders the item's queries by their first time key with a counting sort in LDS (perm),
//    so that the queries of a wave read one or two keys' grid window, which stays in L1/L2;
//  * runs the two-phase query decode over the queries in that order.
// Grid-node window of a tile along one axis: every node that a query binned to texels
// [t0, t0 + TS) can read, i.e. [floor(qlo), floor(qhi) + 1] for the grid positions
// q = (p + 0.5) G / S - 0.5 of the texel positions p in [t0, t0 + TS), widened by 0.01 node
// against rounding and clamped to the grid.  Queries clamped to the map's edge read edge
// nodes, which the clamp keeps inside.  The same arithmetic runs on the host for the
// largest window (kept unfused there and here).
__host__ __device__ __forceinline__ void node_window(int t0, int TS, int S, int G, int& lo, int& hi) {
#pragma clang fp contract(off)
  const float r = (float)G / (float)S;
  const float qlo = ((float)t0 + 0.5f) * r - 0.5f;
  const float qhi = ((float)(t0 + TS) + 0.5f) * r - 0.5f;
  lo = max((int)floorf(qlo - 0.01f), 0);
  hi = min((int)floorf(qhi + 0.01f) + 1, G - 1);
}

constexpr int kGridLdsBytes = 40 * 1024;   // LDS for a tile's grid window over all keys

// Item order: workgroups are dispatched to the 8 XCDs round-robin, so workgroup ids
// x, x+8, ... share one L2.  Each XCD takes one contiguous eighth of the items (tiles in
// row-major order), so tiles processed side by side on an XCD share their halo lines in
// its L2.  Small grids take items round-robin.
struct ItemWalk {
  int first, end, step;
};
__device__ __forceinline__ ItemWalk item_walk(int n_items) {
  ItemWalk w;
  if ((gridDim.x & 7) == 0 && n_items >= (int)gridDim.x) {
    const int chunk = (n_items + 7) >> 3, xcd = blockIdx.x & 7;
    w.first = xcd * chunk + ((int)blockIdx.x >> 3);
    w.end = min(n_items, (xcd + 1) * chunk);
    w.step = gridDim.x >> 3;
  } else {
    w.first = blockIdx.x;
    w.end = n_items;
    w.step = gridDim.x;
  }
  return w;
}

// Tile and query range of one work item.
struct Item {
  int64_t s_lo;     // first sorted query
  int cnt;          // queries (1..kPiece)
  int tx0, ty0;     // tile origin in texels
};
template <int TSL>
__device__ __forceinline__ Item item_at(int it, const BinGeom& bg, const int32_t* __restrict__ start,
                                        const int32_t* __restrict__ items, const int32_t* __restrict__ item_bin) {
  const int b = item_bin[it];
  Item I;
  I.s_lo = (int64_t)start[b] + (int64_t)(it - items[b]) * kPiece;
  I.cnt = (int)(min((int64_t)start[b + 1], I.s_lo + kPiece) - I.s_lo);
  I.tx0 = (b % bg.ntx) << TSL;
  I.ty0 = (b / bg.ntx) << TSL;
  return I;
}

// Decoded spatial texels of the footprint (fx, fy) of a region, row pair rp, from its 64
// block bytes: both rows, 8 bytes per texel (channel c in byte c), written to the region.
template <int R>
__device__ __forceinline__ void region_rows(uint2* reg, const uint4 blk[4], int fx, int fy, int rp) {
  uint32_t r0[8], r1[8];
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    bc4_rows(blk[h].x, blk[h].y, rp, r0[2 * h], r1[2 * h]);
    bc4_rows(blk[h].z, blk[h].w, rp, r0[2 * h + 1], r1[2 * h + 1]);
  }
#pragma unroll
  for (int rr = 0; rr < 2; ++rr) {
    const uint32_t* r = rr ? r1 : r0;
    uint32_t lo4[4], hi4[4];
    transpose4(r[0], r[1], r[2], r[3], lo4);
    transpose4(r[4], r[5], r[6], r[7], hi4);
    uint4* d = (uint4*)(reg + (4 * fy + 2 * rp + rr) * R + 4 * fx);
    d[0] = make_uint4(lo4[0], hi4[0], lo4[1], hi4[1]);
    d[1] = make_uint4(lo4[2], hi4[2], lo4[3], hi4[3]);
  }
}

// One pass of 64 sorted queries of a wave: two-phase decode, RGB to the original index.
template <int PREC, int GDT, int R, typename GridFn>
__device__ __forceinline__ void binned_pass(const Dec<PREC>& dec, const ndgi_model& m, const uint2* reg, int tx0,
                                            int ty0, const float4& rec, bool live, GridFn grid, void* out) {
  float sp[8], gr[8];
  spatial8_lds(reg, R, tx0, ty0, coord_axis(rec.x, m.W), coord_axis(rec.y, m.H), sp);
  grid(rec, gr);
  const f4v acc = decode_regs<PREC>(dec, sp, gr);
  if (live)
    store_rgb<PREC>(out, (size_t)__builtin_bit_cast(uint32_t, rec.w), acc,
                    !(isfinite(rec.x) && isfinite(rec.y) && isfinite(rec.z)));
}

// Decode of the sorted queries with the grid read from HBM (windows too large for LDS, or
// 64-texel tiles).  Per work item the workgroup decodes the tile region into LDS (R = TS + 4
// texels a side: the tile plus one footprint of halo, 8 bytes per texel), orders the
// item's queries by their first time key with a counting sort in LDS (perm), so that a
// wave's queries read one or two keys' grid window from cache, and runs the passes.
template <int PREC, int TSL>
constexpr int binned_waves() { return (PREC == NDGI_PREC_F16 && TSL == 5) ? 4 : 1; }

template <int PREC, int GDT, int TSL>
__global__ __launch_bounds__(256, (binned_waves<PREC, TSL>())) void k_decode_binned(
    ndgi_model m, BinGeom bg, const float4* __restrict__ sorted, const int32_t* __restrict__ start,
    const int32_t* __restrict__ items, const int32_t* __restrict__ item_bin, void* __restrict__ out) {
  constexpr int TS = 1 << TSL;
  constexpr int R = TS + 4;
  constexpr int FP = R / 4;                      // footprints per region side
  constexpr int kTasks = FP * FP * 2;            // (footprint, row pair)
  __shared__ uint2 reg[R * R];
  __shared__ uint16_t perm[kPiece];
  __shared__ int32_t khist[kMaxKeys];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  Dec<PREC> dec;
  dec.load(m.mlp, m.mlp_dtype, lane);
  const uint32_t bw = (uint32_t)m.W >> 2, bh = (uint32_t)m.H >> 2;
  const ItemWalk walk = item_walk(items[bg.ntx * bg.nty]);
  for (int it = walk.first; it < walk.end; it += walk.step) {
    const Item I = item_at<TSL>(it, bg, start, items, item_bin);
    __syncthreads();     // the previous item's readers of reg, perm and khist are done
    for (int i = threadIdx.x; i < m.T; i += 256) khist[i] = 0;
#pragma unroll 1
    for (int task = threadIdx.x; task < kTasks; task += 256) {
      const int rp = task & 1, f = task >> 1;
      const int fy = f / FP, fx = f - FP * fy;
      const uint32_t gfx = (uint32_t)(I.tx0 >> 2) + fx, gfy = (uint32_t)(I.ty0 >> 2) + fy;
      if (gfx < bw && gfy < bh) {
        const uint4* fp = (const uint4*)(m.bc4 + (gfy * bw + gfx) * 64u);
        const uint4 blk[4] = {fp[0], fp[1], fp[2], fp[3]};
        region_rows<R>(reg, blk, fx, fy, rp);
      }
    }
    __syncthreads();     // khist zeroed
    // keys are recomputed in the scatter pass rather than kept: registers hold the decoder
#pragma unroll 1
    for (int i = threadIdx.x; i < I.cnt; i += 256) atomicAdd(&khist[make_keys(sorted[I.s_lo + i].z, m.T).k0], 1);
    __syncthreads();
    if (wave == 0) wave_exclusive_scan(khist, m.T, lane);
    __syncthreads();
#pragma unroll 1
    for (int i = threadIdx.x; i < I.cnt; i += 256)
      perm[atomicAdd(&khist[make_keys(sorted[I.s_lo + i].z, m.T).k0], 1)] = (uint16_t)i;
    __syncthreads();     // reg and perm complete
    auto record = [&](int i) { return sorted[I.s_lo + perm[min(i, I.cnt - 1)]]; };
    float4 next = record(64 * wave + lane);
    for (int p0 = 64 * wave; p0 < I.cnt; p0 += 256) {
      const float4 rec = next;
      if (p0 + 256 < I.cnt) next = record(p0 + 256 + lane);
      binned_pass<PREC, GDT, R>(dec, m, reg, I.tx0, I.ty0, rec, p0 + lane < I.cnt,
                                [&](const float4& q, float* gr) { query_grid8<GDT>(m, q.x, q.y, q.z, gr); }, out);
    }
  }
}

// Grid-node window of a tile (both axes).
struct Win {
  int x0, y0, nx, ny;
};
template <int TS>
__device__ __forceinline__ Win tile_window(const ndgi_model& m, const BinGeom& bg, const Item& I) {
  Win w;
  if (bg.galign) {   // nodes 8k..8k+8 (tile origin 32k texels)
    w.x0 = I.tx0 >> 2;
    w.y0 = I.ty0 >> 2;
    w.nx = min(9, m.Gw - w.x0);
    w.ny = min(9, m.Gh - w.y0);
    return w;
  }
  int x1, y1;
  node_window(I.tx0, TS, m.W, m.Gw, w.x0, x1);
  node_window(I.ty0, TS, m.H, m.Gh, w.y0, y1);
  w.nx = x1 - w.x0 + 1;
  w.ny = y1 - w.y0 + 1;
  return w;
}

constexpr int kWinU4 = kGridLdsBytes / 16;
constexpr int kWinPer = kWinU4 / 256;          // window uint4 per thread
// staging registers use native vectors (arrays of HIP's uint4 wrapper stay in scratch)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Issue this thread's loads for an item: its share of the grid window (node-major over
// keys, rows, columns), the 64 bytes of its region footprint, and its wave's first record.
template <int GDT, int FP, int kTasks>
__device__ __forceinline__ void stage_fetch(const ndgi_model& m, const Item& I, const Win& w,
                                            const float4* __restrict__ sorted, u32x4 (&wv)[kWinPer],
                                            u32x4 (&blk)[4], float4& rec0, int fx, int fy, int wave, int lane) {
  constexpr int kNodeU4 = GDT == NDGI_DTYPE_F16 ? 1 : 2;
  constexpr uint32_t kStep = 256 / kNodeU4;          // window nodes per round of the workgroup
  const u32x4* gsrc = (const u32x4*)m.grid;
  const int total = m.T * w.ny * w.nx * kNodeU4;   // the host checked total <= kWinU4
  // Node nd of the window is (key, rem) = (nd / A, nd % A) with A nodes per key, and rem is
  // (row, column) = (rem / nx, rem % nx).  The thread's first node is divided once; each
  // round then advances (key, rem) by the uniform (dq, dr) with one carry, and rem / nx is
  // (rem * mx) >> 20 with mx = ceil(2^20 / nx), exact while ny * nx^2 <= 2^20 (the host
  // checks this for the largest window).  All products are of 24-bit operands.
  const uint32_t A = (uint32_t)(w.ny * w.nx), nx = (uint32_t)w.nx;
  const uint32_t dq = kStep / A, dr = kStep - dq * A;
  const uint32_t mx = ((1u << 20) + nx - 1) / nx;
  const uint32_t plane = (uint32_t)m.Gh * (uint32_t)m.Gw;
  const uint32_t nd0 = threadIdx.x / kNodeU4, part = threadIdx.x % kNodeU4;
  const uint32_t key0 = nd0 / A;
  uint32_t rem = nd0 - key0 * A, kbase = key0 * plane;   // the key's first node in the grid
  const uint32_t corner = (uint32_t)w.y0 * (uint32_t)m.Gw + (uint32_t)w.x0;
#pragma unroll
  for (int k = 0; k < kWinPer; ++k) {
    const uint32_t gy = __umul24(rem, mx) >> 20, gx = rem - __umul24(gy, nx);
    // threads past the window load its first node (in bounds; nothing is stored for them)
    const uint32_t node = (int)threadIdx.x + 256 * k < total
                              ? kbase + corner + __umul24(gy, (uint32_t)m.Gw) + gx
                              : corner;
    wv[k] = gsrc[node * kNodeU4 + part];
    rem += dr;
    kbase += dq * plane;
    if (rem >= A) {
      rem -= A;
      kbase += plane;
    }
  }
  const uint32_t bw = (uint32_t)m.W >> 2, bh = (uint32_t)m.H >> 2;
  const uint32_t gfx = min((uint32_t)(I.tx0 >> 2) + fx, bw - 1), gfy = min((uint32_t)(I.ty0 >> 2) + fy, bh - 1);
  const u32x4* fp = (const u32x4*)(m.bc4 + (gfy * bw + gfx) * 64u);
#pragma unroll
  for (int h = 0; h < 4; ++h) blk[h] = fp[h];
  rec0 = sorted[I.s_lo + min(64 * wave + lane, I.cnt - 1)];
}

// Write the staged item to LDS: the grid window, and the decoded region rows of this
// thread's task (tasks whose footprint lies outside the map write nothing).
template <int GDT, int R, int kTasks>
__device__ __forceinline__ void stage_commit(const ndgi_model& m, const Item& I, const Win& w,
                                             const u32x4 (&wv)[kWinPer], const u32x4 (&blk)[4], u32x4* gwin,
                                             uint2* reg, int fx, int fy, int rp) {
  constexpr int kNodeU4 = GDT == NDGI_DTYPE_F16 ? 1 : 2;
  const int total = m.T * w.ny * w.nx * kNodeU4;
#pragma unroll
  for (int k = 0; k < kWinPer; ++k) {
    const int idx = (int)threadIdx.x + 256 * k;
    if (idx < total) gwin[idx] = wv[k];
  }
  const uint32_t gfx = (uint32_t)(I.tx0 >> 2) + fx, gfy = (uint32_t)(I.ty0 >> 2) + fy;
  if ((int)threadIdx.x < kTasks && gfx < ((uint32_t)m.W >> 2) && gfy < ((uint32_t)m.H >> 2)) {
    const uint4 b4[4] = {make_uint4(blk[0].x, blk[0].y, blk[0].z, blk[0].w),
                         make_uint4(blk[1].x, blk[1].y, blk[1].z, blk[1].w),
                         make_uint4(blk[2].x, blk[2].y, blk[2].z, blk[2].w),
                         make_uint4(blk[3].x, blk[3].y, blk[3].z, blk[3].w)};
    region_rows<R>(reg, b4, fx, fy, rp);
  }
}

// Decode of the sorted queries with the tile's grid window (all keys) staged in LDS, for
// 32-texel tiles whose window fits kGridLdsBytes.  Per item the workgroup stages the window
// and the decoded region (each thread's loads issued together, then written to LDS); the
// query loop then reads only its records from HBM.  With about 50 KB of LDS, three
// workgroups share a CU, so one workgroup's staging overlaps the others' decoding.
template <int PREC, int GDT>
__global__ __launch_bounds__(256) void k_decode_binned_lds(
    ndgi_model m, BinGeom bg, const float4* __restrict__ sorted, const int32_t* __restrict__ start,
    const int32_t* __restrict__ items, const int32_t* __restrict__ item_bin, void* __restrict__ out) {
  constexpr int TSL = 5, TS = 32, R = TS + 4, FP = R / 4;
  constexpr int kTasks = FP * FP * 2;            // (footprint, row pair): 162 <= 256 threads
  static_assert(kTasks <= 256, "one region task per thread");
  constexpr int kNodeU4 = GDT == NDGI_DTYPE_F16 ? 1 : 2;   // uint4 per grid node
  __shared__ uint2 reg[R * R];
  __shared__ u32x4 gwin[kWinU4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  Dec<PREC> dec;
  dec.load(m.mlp, m.mlp_dtype, lane);
  const ItemWalk walk = item_walk(items[bg.ntx * bg.nty]);
  // this thread's region task
  const int rp = threadIdx.x & 1, f = threadIdx.x >> 1;
  const int fy = f / FP, fx = f - FP * fy;
  for (int it = walk.first; it < walk.end; it += walk.step) {
    const Item I = item_at<TSL>(it, bg, start, items, item_bin);
    const Win w = tile_window<TS>(m, bg, I);
    u32x4 wv[kWinPer], blk[4];
    float4 rec;
    __syncthreads();     // the previous item's readers of reg and gwin are done
    stage_fetch<GDT, FP, kTasks>(m, I, w, sorted, wv, blk, rec, fx, fy, wave, lane);
    stage_commit<GDT, R, kTasks>(m, I, w, wv, blk, gwin, reg, fx, fy, rp);
    __syncthreads();     // reg and gwin complete
    for (int p0 = 64 * wave; p0 < I.cnt; p0 += 256) {
      const float4 cur = rec;
      if (p0 + 256 < I.cnt) rec = sorted[I.s_lo + min(p0 + 256 + lane, I.cnt - 1)];
      // window-local node; the clamp only guards the LDS bounds
      binned_pass<PREC, GDT, R>(dec, m, reg, I.tx0, I.ty0, cur, p0 + lane < I.cnt,
                                [&](const float4& q, float* gr) {
                                  query_grid8_at<GDT>(m, q.x, q.y, q.z, [&](int key, int gy, int gx) {
                                    const int ly = min(max(gy - w.y0, 0), w.ny - 1);
                                    const int lx = min(max(gx - w.x0, 0), w.nx - 1);
                                    const uint32_t nd = __umul24(__umul24((uint32_t)key, (uint32_t)w.ny) + (uint32_t)ly,
                                                                 (uint32_t)w.nx) + (uint32_t)lx;
                                    return (const uint4*)&gwin[nd * kNodeU4];
                                  }, gr);
                                }, out);
    }
  }
}

// Largest grid window of any tile of the map, by the kernel's own arithmetic: its width
// and height in nodes (each the largest over the tiles) and its size in uint4.
static int64_t max_window_u4(const ndgi_model& m, const BinGeom& bg, int& mx, int& my) {
  const int TS = 1 << bg.ts_log2;
  const int64_t node_u4 = m.grid_dtype == NDGI_DTYPE_F16 ? 1 : 2;
  if (bg.galign) {
    mx = std::min(9, m.Gw);
    my = std::min(9, m.Gh);
  } else {
    int lo, hi;
    mx = my = 0;
    for (int t = 0; t < bg.ntx; ++t) {
      node_window(t * TS, TS, m.W, m.Gw, lo, hi);
      mx = std::max(mx, hi - lo + 1);
    }
    for (int t = 0; t < bg.nty; ++t) {
      node_window(t * TS, TS, m.H, m.Gh, lo, hi);
      my = std::max(my, hi - lo + 1);
    }
  }
  return (int64_t)mx * my * m.T * node_u4;
}

struct BinnedLayout {
  BinGeom bg;
  int nbins;
  int64_t max_items;
  int64_t counts_off, start_off, items_off, item_bin_off, bsum_off, sorted_off, bytes;
};

static int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

static bool binned_layout(const ndgi_model& m, int64_t n, BinnedLayout& L) {
  if (!bin_geom(m, L.bg)) return false;
  L.nbins = L.bg.ntx * L.bg.nty;
  L.counts_off = 0;
  L.start_off = align256((int64_t)kSortWgs * L.nbins * 4);
  L.items_off = L.start_off + align256((int64_t)(L.nbins + 1) * 4);
  // at most one item per kPiece queries plus one per bin
  L.max_items = n / kPiece + L.nbins;
  L.item_bin_off = L.items_off + align256((int64_t)(L.nbins + 1) * 4);
  L.bsum_off = L.item_bin_off + align256(L.max_items * 4);
  L.sorted_off = L.bsum_off + align256((int64_t)(kMaxBins / kColBins) * 2 * 4);   // column-scan sums
  L.bytes = L.sorted_off + n * 16;
  return true;
}

bool binned_route(const ndgi_model& m, int64_t n, int64_t ws_bytes) {
  BinnedLayout L;
  if (n <= 0 || n > INT32_MAX || !binned_layout(m, n, L)) return false;
  return n >= kRouteQueriesPerTile * L.nbins && L.bytes <= ws_bytes;
}

int binned_workspace(const ndgi_model& m, int64_t n, int64_t* bytes) {
  BinnedLayout L;
  if (!binned_layout(m, n, L))
    return fail(NDGI_ERR_UNSUPPORTED, "decode_binned: maps above %d tiles of 64x64 texels are not binned",
                kMaxBins);
  *bytes = L.bytes;
  return NDGI_OK;
}

int launch_decode_binned(ndgi_ctx* ctx, const ndgi_model& m, const float* uvt, int64_t n, void* out, int prec,
                         void* ws, int64_t ws_bytes, hipStream_t s) {
  BinnedLayout L;
  if (!binned_layout(m, n, L))
    return fail(NDGI_ERR_UNSUPPORTED, "decode_binned: maps above %d tiles of 64x64 texels are not binned",
                kMaxBins);
  if (ws_bytes < L.bytes)
    return fail(NDGI_ERR_INVALID_ARG, "decode_binned: workspace of %lld bytes, %lld needed", (long long)ws_bytes,
                (long long)L.bytes);
  if ((uintptr_t)ws % 256) return fail(NDGI_ERR_INVALID_ARG, "decode_binned: workspace not 256-byte aligned");
  int32_t* counts = (int32_t*)((char*)ws + L.counts_off);
  int32_t* start = (int32_t*)((char*)ws + L.start_off);
  int32_t* items = (int32_t*)((char*)ws + L.items_off);
  int32_t* item_bin = (int32_t*)((char*)ws + L.item_bin_off);
  int32_t* bsum = (int32_t*)((char*)ws + L.bsum_off);
  float4* sorted = (float4*)((char*)ws + L.sorted_off);
  const int64_t slice = (n + kSortWgs - 1) / kSortWgs;
  hipLaunchKernelGGL(k_bin_count, dim3(kSortWgs), dim3(kSortThreads), 0, s, m, L.bg, uvt, n, slice, counts);
  hipLaunchKernelGGL(k_bin_colscan, dim3((L.nbins + kColBins - 1) / kColBins), dim3(256), 0, s, counts, L.nbins, start,
                     bsum);
  hipLaunchKernelGGL(k_bin_starts, dim3((L.nbins + kStartBins - 1) / kStartBins), dim3(kStartBins), 0, s, start, items,
                     item_bin, L.nbins, (int32_t)n, bsum);
  hipLaunchKernelGGL(k_bin_scatter, dim3(kSortWgs), dim3(kSortThreads), 0, s, m, L.bg, uvt, n, slice, counts, start,
                     sorted);
  NDGI_HIP(hipGetLastError());
  const bool g16 = m.grid_dtype == NDGI_DTYPE_F16;
  // grid window in LDS when it fits (32-texel tiles only)
  // (the staging's row split (rem * mx) >> 20 is exact while ny * nx^2 <= 2^20)
  int wmx, wmy;
  const int64_t win_u4 = max_window_u4(m, L.bg, wmx, wmy);
  const bool glds = L.bg.ts_log2 == 5 && win_u4 * 16 <= kGridLdsBytes && (int64_t)wmy * wmx * wmx <= (1 << 20);
#define NDGI_BINNED_KERNEL(K)                                                                             \
  do {                                                                                                    \
    int64_t wgs = resident_wgs(ctx, (const void*)K);                                                      \
    if (wgs > L.max_items) wgs = L.max_items;                                                             \
    hipLaunchKernelGGL(K, dim3((unsigned)wgs), dim3(256), 0, s, m, L.bg, sorted, start, items, item_bin, out); \
  } while (0)
#define NDGI_BINNED_TS(P, G)                                              \
  do {                                                                    \
    if (glds) NDGI_BINNED_KERNEL((k_decode_binned_lds<P, G>));            \
    else if (L.bg.ts_log2 == 5) NDGI_BINNED_KERNEL((k_decode_binned<P, G, 5>)); \
    else NDGI_BINNED_KERNEL((k_decode_binned<P, G, 6>));                  \
  } while (0)
  if (prec == NDGI_PREC_F16) {
    if (g16) NDGI_BINNED_TS(NDGI_PREC_F16, NDGI_DTYPE_F16);
    else NDGI_BINNED_TS(NDGI_PREC_F16, NDGI_DTYPE_F32);
  } else {
    if (g16) NDGI_BINNED_TS(NDGI_PREC_F32, NDGI_DTYPE_F16);
    else NDGI_BINNED_TS(NDGI_PREC_F32, NDGI_DTYPE_F32);
  }
#undef NDGI_BINNED_TS
#undef NDGI_BINNED_KERNEL
  NDGI_HIP(hipGetLastError());
  return NDGI_OK;
}

}  // namespace ndgi
