// demod stage: max-log LLRs, one thread per (frame, user, subcarrier) looping
// over the data symbols (consecutive threads write consecutive LLR groups of
// one symbol row).  The body is demk::demod_column; frames are contiguous, so
// the frame index folds into the user index.
#include "demod_core.h"

namespace rxphy {
namespace {

using namespace demk;

template <int Q>
__global__ void __launch_bounds__(256)
demod_kernel(const float2* __restrict__ xt, const float* __restrict__ nu, float* __restrict__ llr,
             int D, int n_sc) {
  const int i = blockIdx.x * 256 + tid_x();
  if (i >= n_sc) return;
  const int64_t fu = blockIdx.y;                  // frame * K + user (offset by the launcher)
  demod_column<Q>(xt + fu * D * n_sc + i, nu[fu * n_sc + i], llr + (fu * D * n_sc + i) * Q, D, n_sc);
}

// Downlink QAM mapping, four points per thread: bits [n][Q] (one byte each,
// b0 first; any non-zero byte is a one) -> the Gray point with that label,
// each axis from the same level table as the demapper.  With a 4-byte aligned
// bits pointer and a 16-byte aligned output a thread reads its 4Q bytes as Q
// words and writes two 16-byte pairs; otherwise (and for the ragged tail) it
// reads byte by byte.
template <int Q>
__device__ __forceinline__ float2 map_point(int ci, int cq) {
  return make_float2(axis_level<Q>(ci), axis_level<Q>(cq));
}

template <int Q>
__global__ void __launch_bounds__(256)
modulate_kernel(const uint8_t* __restrict__ bits, float2* __restrict__ sym, int64_t n, int vec) {
  const int64_t p0 = 4 * ((int64_t)blockIdx.x * 256 + threadIdx.x);
  if (p0 >= n) return;
  if (vec && p0 + 4 <= n) {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(bits + p0 * Q);
    uint32_t wd[Q];
#pragma unroll
    for (int k = 0; k < Q; ++k) wd[k] = src[k];
    float2 pt[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      int ci = 0, cq = 0;                         // axis codes: b0 b2 b4 / b1 b3 b5, MSB first
#pragma unroll
      for (int t = 0; t < Q / 2; ++t) {
        const int e = j * Q + 2 * t;              // byte index of b_{2t} of point j
        ci = 2 * ci + (((wd[e >> 2] >> (8 * (e & 3))) & 0xffu) != 0);
        cq = 2 * cq + (((wd[(e + 1) >> 2] >> (8 * ((e + 1) & 3))) & 0xffu) != 0);
      }
      pt[j] = map_point<Q>(ci, cq);
    }
    float4* o = reinterpret_cast<float4*>(sym + p0);
    o[0] = make_float4(pt[0].x, pt[0].y, pt[1].x, pt[1].y);
    o[1] = make_float4(pt[2].x, pt[2].y, pt[3].x, pt[3].y);
    return;
  }
  const int64_t pe = p0 + 4 < n ? p0 + 4 : n;
  for (int64_t p = p0; p < pe; ++p) {
    const uint8_t* b = bits + p * Q;
    int ci = 0, cq = 0;
#pragma unroll
    for (int t = 0; t < Q / 2; ++t) {
      ci = 2 * ci + (b[2 * t] != 0);
      cq = 2 * cq + (b[2 * t + 1] != 0);
    }
    sym[p] = map_point<Q>(ci, cq);
  }
}

}  // namespace

rxphy_status launch_modulate(const rxphy_frame& fr, int64_t n_points, const uint8_t* bits, float2* sym,
                             hipStream_t s) {
  if (n_points == 0) return RXPHY_OK;
  const int64_t blocks = (n_points + 1023) / 1024;
  if (blocks > 0x7fffffff) return fail(RXPHY_EUNSUPPORTED, "too many points (%lld)", (long long)n_points);
  const int vec = ((uintptr_t)bits & 3u) == 0 && ((uintptr_t)sym & 15u) == 0;
  const dim3 grid((unsigned)blocks);
  switch (fr.qam_bits) {
    case 2: hipLaunchKernelGGL(modulate_kernel<2>, grid, dim3(256), 0, s, bits, sym, n_points, vec); break;
    case 4: hipLaunchKernelGGL(modulate_kernel<4>, grid, dim3(256), 0, s, bits, sym, n_points, vec); break;
    case 6: hipLaunchKernelGGL(modulate_kernel<6>, grid, dim3(256), 0, s, bits, sym, n_points, vec); break;
    default: return fail(RXPHY_EINVAL, "qam_bits = %d", fr.qam_bits);
  }
  return launch_status("modulate kernel");
}

rxphy_status launch_demod(const rxphy_frame& fr, int32_t nf, const float2* xt, const float* nu,
                          float* llr, hipStream_t s) {
  const int D = fr.n_sym - 1;
  const int64_t cols = (int64_t)nf * fr.K;        // (frame, user) rows, 65535 per launch
  const unsigned bx = (unsigned)((fr.n_sc + 255) / 256);
  for (int64_t c0 = 0; c0 < cols; c0 += 65535) {
    const unsigned by = (unsigned)(cols - c0 < 65535 ? cols - c0 : 65535);
    const float2* x0 = xt + c0 * D * fr.n_sc;
    const float* v0 = nu + c0 * fr.n_sc;
    float* l0 = llr + c0 * D * fr.n_sc * fr.qam_bits;
    switch (fr.qam_bits) {
      case 2: hipLaunchKernelGGL(demod_kernel<2>, dim3(bx, by), dim3(256), 0, s, x0, v0, l0, D, fr.n_sc); break;
      case 4: hipLaunchKernelGGL(demod_kernel<4>, dim3(bx, by), dim3(256), 0, s, x0, v0, l0, D, fr.n_sc); break;
      case 6: hipLaunchKernelGGL(demod_kernel<6>, dim3(bx, by), dim3(256), 0, s, x0, v0, l0, D, fr.n_sc); break;
      default: return fail(RXPHY_EINVAL, "qam_bits = %d", fr.qam_bits);
    }
    rxphy_status st = launch_status("demod kernel");
    if (st) return st;
  }
  return RXPHY_OK;
}

}  // namespace rxphy
