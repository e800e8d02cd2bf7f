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
template <int Q>
__device__ __forceinline__ void axis_llr(float x, float inv_nu, float* out) {
  constexpr int B = Q / 2;
  constexpr int NL = 1 << B;
  float d0[B], d1[B], l0[B], l1[B];
#pragma unroll
  for (int t = 0; t < B; ++t) { d0[t] = d1[t] = INFINITY; l0[t] = l1[t] = 0.f; }
#pragma unroll
  for (int code = 0; code < NL; ++code) {   // increasing code = increasing point index
    const float lv = axis_level<Q>(code);
    const float d = (x - lv) * (x - lv);
#pragma unroll
    for (int t = 0; t < B; ++t) {
      const bool one = (code >> (B - 1 - t)) & 1;
      if (one) { if (d < d1[t]) { d1[t] = d; l1[t] = lv; } }
      else     { if (d < d0[t]) { d0[t] = d; l0[t] = lv; } }
    }
  }
#pragma unroll
  for (int t = 0; t < B; ++t) out[t] = (l0[t] - l1[t]) * (2.f * x - l0[t] - l1[t]) * inv_nu;
}


// LLRs of one equalised symbol x with noise variance v (erased when v = inf)
// into dst[0 .. Q-1]; STREAM: store with the non-temporal hint (measured: it
// helps the fused detector, whose LLR stream competes with its data loads,
// and slows the demod stage's own kernel).
template <int Q, bool STREAM = false>
__device__ __forceinline__ void demod_point(float2 x, float v, float* __restrict__ dst) {
  float o[Q];
  if (__builtin_isinf(v)) {
#pragma unroll
    for (int j = 0; j < Q; ++j) o[j] = 0.f;
  } else {
    const float inv = 1.0f / v;
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

// One (user, subcarrier) column: xc = &x_tilde[u][0][i], lc = &llr[u][0][i][0];
// nu is read once and the D data symbols are demapped CH loads at a time
// (more loads in flight per thread where fewer waves are resident).
template <int Q, int CH = 4>
__device__ __forceinline__ void demod_column(const float2* __restrict__ xc, float v,
                                             float* __restrict__ lc, int D, int n_sc) {
  int d = 0;
  for (; d + CH <= D; d += CH) {
    float2 x[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) x[k] = xc[(uint32_t)(d + k) * n_sc];
#pragma unroll
    for (int k = 0; k < CH; ++k) demod_point<Q>(x[k], v, lc + (uint32_t)(d + k) * n_sc * Q);
  }
  for (; d < D; ++d) demod_point<Q>(xc[(uint32_t)d * n_sc], v, lc + (uint32_t)d * n_sc * Q);
}

}  // namespace demk
}  // namespace rxphy
