// Max-log LLR body over the Gray square-QAM set, shared by the per-stage
// demod kernel and the persistent batched kernel.
//
// The constellation is the Cartesian product of two Gray PAM axes (b0, b2, b4
// on the in-phase axis, b1, b3, b5 on the quadrature axis), so for a bit on one
// axis the other axis contributes the same minimum to both sides and cancels:
// each LLR is an exact max-log value computed from one axis alone,
//   llr = ((x - l1)^2 - (x - l0)^2) / nu = (l0 - l1)(2x - l0 - l1) / nu,
// with l_b the nearest level whose bit is b (the product form avoids the
// cancellation of the two squares).
#pragma once

#include "common.h"

namespace rxphy {
namespace demk {

template <int Q>
__device__ __forceinline__ float axis_level(int code) {
  // code bit (B-1-t) is the axis' t-th bit; t = 0 is the sign bit
  constexpr int B = Q / 2;
  if constexpr (B == 1) {
    return (code & 1) ? -0.70710678118654752f : 0.70710678118654752f;
  } else if constexpr (B == 2) {
    const float s0 = (code & 2) ? -1.f : 1.f, s1 = (code & 1) ? -1.f : 1.f;
    return s0 * (2.f - s1) * 0.31622776601683793f;      // 1/sqrt(10)
  } else {
    const float s0 = (code & 4) ? -1.f : 1.f, s1 = (code & 2) ? -1.f : 1.f, s2 = (code & 1) ? -1.f : 1.f;
    return s0 * (4.f - s1 * (2.f - s2)) * 0.15430334996209191f;   // 1/sqrt(42)
  }
}

// LLRs of the B bits carried by one axis at coordinate x (out[t] for axis bit t).
// The levels are c times the odd integers -(2^B - 1) .. 2^B - 1, and each bit
// splits them into two sets whose nearest member follows in closed form from
// the nearest odd integer o to x / c (ties go up; the LLR is the same on both
// sides of a tie):
//   sign bit:        0 -> {+1, .., +(2^B-1)}  clamp(o, 1, 2^B-1);  1 -> the mirror image
//   16-QAM bit 1:    0 -> |level| 1           +-1 by the sign of o; 1 -> +-3
//   64-QAM bit 1:    0 -> |level| in {1, 3}   clamp(o, -3, 3);     1 -> +-clamp(|o|, 5, 7)
//   64-QAM bit 2:    0 -> |level| in {3, 5}   +-clamp(|o|, 3, 5);  1 -> +-(|o| < 4 ? 1 : 7)
// (the magnitudes of axis_level: 2 - s1 and 4 - s1 (2 - s2)).  The chosen
// levels are those of a search over all 2^B levels except within rounding of
// a midpoint, and a huge |x| keeps its large LLR (a search would square it to
// infinity).
template <int Q>
__device__ __forceinline__ void axis_llr(float x, float inv_nu, float* out) {
  constexpr int B = Q / 2;
  float l0[B], l1[B];
  if constexpr (B == 1) {
    l0[0] = 0.70710678118654752f;
    l1[0] = -0.70710678118654752f;
  } else {
    constexpr float c = B == 2 ? 0.31622776601683793f : 0.15430334996209191f;   // 1/sqrt(10), 1/sqrt(42)
    constexpr float ic = B == 2 ? 3.16227766016837933f : 6.48074069840786023f;  // sqrt(10), sqrt(42)
    const float o = 2.f * __builtin_floorf(0.5f * (x * ic)) + 1.f;
    auto clampf = [](float v, float lo, float hi) { return __builtin_fminf(__builtin_fmaxf(v, lo), hi); };
    if constexpr (B == 2) {
      l0[0] = clampf(o, 1.f, 3.f);
      l1[0] = clampf(o, -3.f, -1.f);
      l0[1] = clampf(o, -1.f, 1.f);
      l1[1] = __builtin_copysignf(3.f, o);
    } else {
      const float m = __builtin_fabsf(o);
      l0[0] = clampf(o, 1.f, 7.f);
      l1[0] = clampf(o, -7.f, -1.f);
      l0[1] = clampf(o, -3.f, 3.f);
      l1[1] = __builtin_copysignf(clampf(m, 5.f, 7.f), o);
      l0[2] = __builtin_copysignf(clampf(m, 3.f, 5.f), o);
      l1[2] = __builtin_copysignf(m < 4.f ? 1.f : 7.f, o);
    }
#pragma unroll
    for (int t = 0; t < B; ++t) {
      l0[t] *= c;
      l1[t] *= c;
    }
  }
#pragma unroll
  for (int t = 0; t < B; ++t) out[t] = (l0[t] - l1[t]) * (2.f * x - l0[t] - l1[t]) * inv_nu;
}

// LLRs of one equalised symbol x into dst[0 .. Q-1], erased (all zero) or
// with inv = 1 / v formed by the caller; STREAM: store with the non-temporal
// hint (measured: it helps the fused detector, whose LLR stream competes with
// its data loads, and slows the demod stage's own kernel).
template <int Q, bool STREAM = false>
__device__ __forceinline__ void demod_point_inv(float2 x, bool erased, float inv, float* __restrict__ dst) {
  float o[Q];
  if (erased) {
#pragma unroll
    for (int j = 0; j < Q; ++j) o[j] = 0.f;
  } else {
    float re[Q / 2], im[Q / 2];
    axis_llr<Q>(x.x, inv, re);
    axis_llr<Q>(x.y, inv, im);
#pragma unroll
    for (int t = 0; t < Q / 2; ++t) { o[2 * t] = re[t]; o[2 * t + 1] = im[t]; }
  }
#pragma unroll
  for (int t = 0; t < Q / 2; ++t) {
    const float2 pr = make_float2(o[2 * t], o[2 * t + 1]);
    if constexpr (STREAM) store_stream2(reinterpret_cast<float2*>(dst) + t, pr);
    else reinterpret_cast<float2*>(dst)[t] = pr;
  }
}

// LLRs of one equalised symbol x with noise variance v (erased when v = inf).
template <int Q, bool STREAM = false>
__device__ __forceinline__ void demod_point(float2 x, float v, float* __restrict__ dst) {
  const bool erased = __builtin_isinf(v);
  demod_point_inv<Q, STREAM>(x, erased, erased ? 0.f : 1.0f / v, dst);
}

// One (user, subcarrier) column: xc = &x_tilde[u][0][i], lc = &llr[u][0][i][0];
// nu is read once and the D data symbols are demapped CH loads at a time
// (more loads in flight per thread where fewer waves are resident).
template <int Q, int CH = 4>
__device__ __forceinline__ void demod_column(const float2* __restrict__ xc, float v,
                                             float* __restrict__ lc, int D, int n_sc) {
  const bool er = __builtin_isinf(v);
  const float inv = er ? 0.f : 1.0f / v;
  int d = 0;
  for (; d + CH <= D; d += CH) {
    float2 x[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) x[k] = xc[(uint32_t)(d + k) * n_sc];
#pragma unroll
    for (int k = 0; k < CH; ++k) demod_point_inv<Q>(x[k], er, inv, lc + (uint32_t)(d + k) * n_sc * Q);
  }
  for (; d < D; ++d) demod_point_inv<Q>(xc[(uint32_t)d * n_sc], er, inv, lc + (uint32_t)d * n_sc * Q);
}

}  // namespace demk
}  // namespace rxphy
