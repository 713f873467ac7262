// Shared pieces of the hybrid-layout kernels (decode and training): packed decoder
// offsets, GELU, and the time axis (key table, node-aligned samples).
#pragma once
#include "device.hpp"

namespace ndgi {

template <int HD>
struct HybShape {
  static constexpr int NB = HD / 16;                           // row blocks of a hidden layer
  static constexpr int kL1 = 0, kL2 = NB, kL3 = NB + NB * NB;  // first chunk of each layer
  static constexpr int kChunks = NB + NB * NB + NB;
  static constexpr int oW1 = 0, oB1 = HD * NDGI_HYBRID_IN, oW2 = oB1 + HD, oB2 = oW2 + HD * HD,
                       oW3 = oB2 + HD, oB3 = oW3 + 3 * HD, kSize = oB3 + 3;
};

// GELU(x) = x Phi(x) = max(x, 0) - |x| * erfc(|x| / sqrt 2) / 2: both signs are the same
// expression, with no cancellation for large |x|.  The factor 1/2 and the argument scale
// 1/sqrt 2 are folded into the constants below.
//  * FP32 path: erfc by the Chebyshev fit of Press et al., Numerical Recipes (erfcc),
//    relative error below 1.2e-7 for every argument: erfc(z) = t exp(-z^2 + p(t)) with
//    t = 1 / (1 + z/2); here exp runs in base 2 with log2(e) folded into p and ln(1/2)
//    added to its constant term;
//  * FP16 path: Q(a) = erfc(a / sqrt 2) / 2 = exp2(p(a)) with a = min(|x|, 6) and p the
//    degree-4 polynomial fitted to log2 Q on [0, 6] by least squares weighted by a Q(a)
//    (the size of the term in GELU); the GELU error stays below 1e-5 for every x (beyond
//    |x| = 6 below 2e-9 |x|), under the FP16 rounding of the activations it feeds (an FP16
//    ulp is 6e-5 at 0.1, where the error peaks): four FMAs and one exponential.
namespace gelu_k {
constexpr double kLog2e = 1.4426950408889634, kRs2 = 0.70710678118654752, kLn2 = 0.69314718055994531;
// Numerical Recipes erfcc coefficients, innermost first, then the constant term
constexpr double kNR[10] = {0.17087277, -0.82215223, 1.48851587, -1.13520398, 0.27886807,
                            -0.18628806, 0.09678418, 0.37409196, 1.00002368, -1.26551223};
// log2(erfc(a / sqrt 2) / 2) ~ sum kQ[i] a^i on [0, 6] (the weighted fit described above)
constexpr float kQ[5] = {-1.00068176e+00f, -1.14647341e+00f, -4.69236821e-01f,
                         -4.34483998e-02f, 3.75886331e-03f};
constexpr float nr_c(int i) { return (float)(kLog2e * (i == 9 ? kNR[9] - kLn2 : kNR[i])); }
// evaluated by the compiler (constexpr variables), never on the device
constexpr float kNRf[10] = {nr_c(0), nr_c(1), nr_c(2), nr_c(3), nr_c(4), nr_c(5), nr_c(6), nr_c(7), nr_c(8), nr_c(9)};
}  // namespace gelu_k

template <int PREC>
__device__ __forceinline__ float gelu(float x) {
  using namespace gelu_k;
  const float ax = fabsf(x);
  float half_erfc;
  if constexpr (PREC == NDGI_PREC_F32) {
    const float t = __builtin_amdgcn_rcpf(fmaf((float)(0.5 * kRs2), ax, 1.0f));
    float p = fmaf(t, kNRf[0], kNRf[1]);
#pragma unroll
    for (int i = 2; i < 10; ++i) p = fmaf(t, p, kNRf[i]);
    half_erfc = t * __builtin_amdgcn_exp2f(fmaf(x * x, (float)(-0.5 * kLog2e), p));
  } else {
    const float a = __builtin_amdgcn_fmed3f(ax, 0.0f, 6.0f);   // min(|x|, 6)
    float p = fmaf(a, kQ[4], kQ[3]);
#pragma unroll
    for (int i = 2; i >= 0; --i) p = fmaf(a, p, kQ[i]);
    half_erfc = __builtin_amdgcn_exp2f(p);
  }
  // max(x, 0) as one median-of-three with the largest float (fmaxf would first quieten
  // signalling NaNs, one more instruction per operand, and a median with +inf is folded
  // back into fmaxf; a non-finite query's output is set to NaN explicitly anyway)
  return fmaf(-ax, half_erfc, __builtin_amdgcn_fmed3f(x, 0.0f, 3.40282347e38f));
}

// GELU and its derivative Phi(x) + x phi(x) for training, in FP32: Phi from the same
// erfc (Phi(x) = erfc(-x / sqrt 2) / 2), phi = exp(-x^2 / 2) / sqrt(2 pi).
__device__ __forceinline__ float gelu_grad(float x) {
  using namespace gelu_k;
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf((float)(0.5 * kRs2), ax, 1.0f));
  float p = fmaf(t, kNRf[0], kNRf[1]);
#pragma unroll
  for (int i = 2; i < 10; ++i) p = fmaf(t, p, kNRf[i]);
  const float e2 = __builtin_amdgcn_exp2f(fmaf(x * x, (float)(-0.5 * kLog2e), 0.0f));   // exp(-x^2 / 2)
  const float half_erfc = t * __builtin_amdgcn_exp2f(fmaf(x * x, (float)(-0.5 * kLog2e), p));
  const float phi_cdf = x >= 0.0f ? 1.0f - half_erfc : half_erfc;
  return fmaf(x, e2 * (float)(0.39894228040143268), phi_cdf);   // 1 / sqrt(2 pi)
}

__device__ __forceinline__ float clamp01(float t) { return fminf(fmaxf(t, 0.0f), 1.0f); }   // NaN -> 0

// Time coordinate tau of a clamped t: piecewise linear through (key_i, i / (n - 1)), clamped
// to [0, 1]; t itself without a key table.  The segment is the last key <= t (within
// [0, n-2]), found by a fixed-step binary search.
template <typename KeyAt>
__device__ __forceinline__ float key_tau(float tc, int n, KeyAt key) {
  if (n < 2) return tc;
  int i = 0;
  for (int step = NDGI_HYBRID_MAX_KEYS / 2; step > 0; step >>= 1) {
    const int j = i + step;
    if (key(min(j, n - 2)) <= tc && j <= n - 2) i = j;   // the read stays inside the table
  }
  const float k0 = key(i), k1 = key(i + 1);
  const float f = (tc - k0) / (k1 - k0);
  return clamp01(((float)i + f) / (float)(n - 1));
}

// Linear interpolation over N samples held at tau = k / (N - 1).
struct NodeT { int i0, i1; float w0, w1; };
__device__ __forceinline__ NodeT node_axis(float tau, int N) {
  NodeT a;
  if (N < 2) {
    a.i0 = a.i1 = 0;
    a.w0 = 1.0f;
    a.w1 = 0.0f;
    return a;
  }
  const float p = tau * (float)(N - 1);
  a.i0 = min((int)floorf(p), N - 2);
  a.i1 = a.i0 + 1;
  a.w1 = p - (float)a.i0;
  a.w0 = 1.0f - a.w1;
  return a;
}

}  // namespace ndgi
