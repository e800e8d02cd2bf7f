// csi stage: least-squares channel estimate from comb pilots, held over the
// pilot group.
//
// Workgroup = one (frame, antenna) and a tile of 512 consecutive subcarriers.
// The LS value Yf0[q] conj(p[q]) / |p[q]|^2 is formed once per pilot
// subcarrier q that the tile needs and parked in LDS; every thread then
// writes two subcarriers of each user's row of H, so each store instruction of
// a wave covers 512 contiguous bytes.
#include "common.h"

namespace rxphy {
namespace {

constexpr int TILE = 512;
constexpr int WG = 256;

__global__ void __launch_bounds__(WG)
csi_kernel(const float2* __restrict__ yf, const float2* __restrict__ pil, float2* __restrict__ h,
           int M, int K, int S, int n_sc) {
  __shared__ float2 ls[TILE + 32];
  const int i0 = blockIdx.x * TILE;
  const int m = blockIdx.y;
  const int f = blockIdx.z;
  const int G = n_sc / K;
  const int i_last = min(i0 + TILE, n_sc) - 1;
  const int q0 = min(i0 / K, G - 1) * K;                     // first pilot subcarrier needed
  const int q1 = min(i_last / K, G - 1) * K + K;             // one past the last
  const float2* y0 = yf + ((int64_t)(f * M + m) * S) * n_sc;
  const float2* pf = pil + (int64_t)f * n_sc;
  for (int q = q0 + threadIdx.x; q < q1; q += WG) {
    const float2 y = y0[q];
    const float2 p = pf[q];
    const float pp = p.x * p.x + p.y * p.y;
    // y conj(p) / |p|^2 ; a zero pilot gives 0/0 = NaN, flagged downstream
    ls[q - q0] = make_float2((y.x * p.x + y.y * p.y) / pp, (y.y * p.x - y.x * p.y) / pp);
  }
  __syncthreads();
  int gq[2];
  bool ok[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const int i = i0 + threadIdx.x + e * WG;
    ok[e] = i < n_sc;
    gq[e] = ok[e] ? min(i / K, G - 1) * K - q0 : 0;
  }
  float2* hm = h + ((int64_t)(f * M + m) * K) * n_sc + i0 + threadIdx.x;
  for (int u = 0; u < K; ++u) {
#pragma unroll
    for (int e = 0; e < 2; ++e)
      if (ok[e]) hm[(int64_t)u * n_sc + e * WG] = ls[gq[e] + u];
  }
}

}  // namespace

rxphy_status launch_csi(const rxphy_frame& fr, int32_t nf, const float2* yf, const float2* pil,
                        float2* h, hipStream_t s) {
  if (nf > 65535) return fail(RXPHY_EUNSUPPORTED, "n_frames = %d > 65535", nf);
  dim3 grid((fr.n_sc + TILE - 1) / TILE, fr.M, nf);
  hipLaunchKernelGGL(csi_kernel, grid, dim3(WG), 0, s, yf, pil, h, fr.M, fr.K, fr.n_sym, fr.n_sc);
  return launch_status("csi kernel");
}

}  // namespace rxphy
